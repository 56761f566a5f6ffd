// Gate-bootstrapping kernels for gfx950: key conversion to the NTT domain, the gate
// prologue (linear combination + modulus switch), blind rotation with SampleExtract,
// identity key switching, and test kernels for the external product and polynomial product.
#include "vsp_internal.h"
#include "blind_rotate.h"
#include "blind_rotate_wide.h"

namespace vsp {

// ------------------------------------------------------------------ key conversion
// One wave per (item, round k, output polynomial c): lanes 0-31 transform TRGSW row k,
// lanes 32-63 row k + 3, both taking column c; results land in the key layout of ntt.h.
__global__ __launch_bounds__(256) void k_trgsw_to_ntt(const u32* __restrict__ src, u64* __restrict__ dst,
                                                      const u64* __restrict__ tw, u64 ninv, uint64_t jobs) {
  __shared__ u32 lds[4 * WAVE_T_U32];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t job = (uint64_t)blockIdx.x * 4 + wave;
  if (job >= jobs) return;
  const int lane = threadIdx.x & 63, l = lane & 31, h = lane >> 5;
  const uint64_t item = job / 6;
  const int rem = (int)(job % 6), k = rem >> 1, c = rem & 1;
  const int row = k + GADGET_L * h;
  const u32* poly = src + ((item * 2 * GADGET_L + row) * 2 + c) * RING_N;
  u64 v[32];
#pragma unroll
  for (int t = 0; t < 32; t++) v[t] = poly[l + 32 * t];
  u32* reg = lds + wave * WAVE_T_U32 + h * TREGION;
  ntt_forward(v, tw, reg, l);
  // lanes 0-31 hold row k, lanes 32-63 row k + 3, both for output polynomial c: they become
  // entries 0 and 1 of lane l + 32 c
  u64* out = dst + item * TRGSW_NTT_U64 + (size_t)k * 32 * 64 * 2;
#pragma unroll
  for (int s = 0; s < 32; s++) out[((size_t)s * 64 + l + 32 * c) * 2 + h] = gl_canon(gl_mul(v[s], ninv));
}

hipError_t launch_trgsw_to_ntt(const vsp_context* ctx, const uint32_t* src, uint64_t* dst, uint64_t count,
                               hipStream_t st) {
  if (count == 0) return hipSuccess;
  const uint64_t jobs = count * 6;
  const u64 ninv = gl_powmod_const(RING_N, GL_P - 2);
  hipLaunchKernelGGL(k_trgsw_to_ntt, dim3((unsigned)((jobs + 3) / 4)), dim3(256), 0, st, src, dst, ctx->tw, ninv,
                     jobs);
  return hipGetLastError();
}

// ------------------------------------------------------------------ gate prologue
// Linear combination of a homomorphic gate on the +-1/8 encoding (standard TFHE gates),
// then modulus switch of every coefficient to Z/2N: round(x 2N / 2^32).
__device__ __forceinline__ bool gate_linear(uint32_t op, u32 x, u32 y, bool is_b, u32& r) {
  const u32 E = MU, Q = 2 * MU;
  switch (op) {
    case VSP_NAND: r = (is_b ? E : 0u) - x - y; return true;
    case VSP_AND: r = (is_b ? 0u - E : 0u) + x + y; return true;
    case VSP_OR: r = (is_b ? E : 0u) + x + y; return true;
    case VSP_NOR: r = (is_b ? 0u - E : 0u) - x - y; return true;
    case VSP_XOR: r = (is_b ? Q : 0u) + 2u * (x + y); return true;
    case VSP_XNOR: r = (is_b ? 0u - Q : 0u) - 2u * (x + y); return true;
    case VSP_ANDNOT: r = (is_b ? 0u - E : 0u) + x - y; return true;
    case VSP_ORNOT: r = (is_b ? E : 0u) + x - y; return true;
    case OP_IDENT: r = x; return true;
    default: return false;
  }
}

__device__ __forceinline__ u32 modswitch_2n(u32 x) { return ((x + (1u << 20)) >> 21) & (2 * RING_N - 1); }

__global__ __launch_bounds__(256) void k_gate_prologue(const uint8_t* __restrict__ ops, uint32_t uniform_op,
                                                       const u32* __restrict__ in0, const u32* __restrict__ in1,
                                                       const u32* __restrict__ idx0, const u32* __restrict__ idx1,
                                                       const u32* __restrict__ idxo, u32* __restrict__ abar,
                                                       u32* __restrict__ out, int* __restrict__ err, uint64_t B,
                                                       int allow_not) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * TLWE0) return;
  const uint64_t g = i / TLWE0;
  const int c = (int)(i - g * TLWE0);
  const uint32_t op = ops ? ops[g] : uniform_op;
  if (op == OP_SKIP) return;
  const uint64_t r0 = idx0 ? idx0[g] : g, r1 = idx1 ? idx1[g] : g;
  const u32 x = in0[r0 * TLWE0 + c];
  const bool one_input = (op == VSP_NOT || op == OP_IDENT || !op_bootstraps(op));
  const u32 y = one_input ? 0u : in1[r1 * TLWE0 + c];
  u32 r;
  if (gate_linear(op, x, y, c == LWE_N, r)) {
    abar[g * TLWE0 + c] = modswitch_2n(r);
  } else if (op == VSP_NOT && allow_not) {
    const uint64_t ro = idxo ? idxo[g] : g;
    out[ro * TLWE0 + c] = 0u - x;
  } else {
    if (out) {
      const uint64_t ro = idxo ? idxo[g] : g;
      out[ro * TLWE0 + c] = 0u;
    }
    if (c == 0) atomicOr(err, DEVERR_BAD_OP);
  }
}

hipError_t launch_gate_prologue(const vsp_context* ctx, const uint8_t* ops, const uint32_t* in0, const uint32_t* in1,
                                const uint32_t* idx0, const uint32_t* idx1, const uint32_t* idxo, uint32_t* abar,
                                uint32_t* out, uint64_t B, hipStream_t st, bool allow_not) {
  if (B == 0) return hipSuccess;
  const uint64_t n = B * TLWE0;
  hipLaunchKernelGGL(k_gate_prologue, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ops, 0u, in0, in1, idx0,
                     idx1, idxo, abar, out, ctx->dev_err, B, allow_not ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_gate_prologue_uniform(const vsp_context* ctx, uint32_t op, const uint32_t* in0, uint32_t* abar,
                                        uint64_t B, hipStream_t st) {
  if (B == 0) return hipSuccess;
  const uint64_t n = B * TLWE0;
  hipLaunchKernelGGL(k_gate_prologue, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nullptr, op, in0, in0,
                     nullptr, nullptr, nullptr, abar, nullptr, ctx->dev_err, B, 0);
  return hipGetLastError();
}

// ------------------------------------------------------------------ homomorphic MUX
// Prologue of s ? c1 : c0 over 2B bootstraps: row g < B takes AND(s, c1), row B + g takes
// ANDNOT(c0, s) (then the modulus switch).
__global__ __launch_bounds__(256) void k_mux_prologue(const u32* __restrict__ sel, const u32* __restrict__ in1,
                                                      const u32* __restrict__ in0, u32* __restrict__ abar,
                                                      uint64_t B) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * B * TLWE0) return;
  const uint64_t r = i / TLWE0;
  const int c = (int)(i - r * TLWE0);
  const bool second = r >= B;
  const uint64_t g = second ? r - B : r;
  const u32 s = sel[g * TLWE0 + c];
  u32 v;
  if (second)
    gate_linear(VSP_ANDNOT, in0[g * TLWE0 + c], s, c == LWE_N, v);
  else
    gate_linear(VSP_AND, s, in1[g * TLWE0 + c], c == LWE_N, v);
  abar[r * TLWE0 + c] = modswitch_2n(v);
}

// t[g] += t[B + g] + (0, ..., 0, mu): the sum of the two extracted halves plus the constant
// term of the HomMUX without SE and IKS (SampleExtract is linear).
__global__ __launch_bounds__(256) void k_mux_combine(u32* __restrict__ t, uint64_t B) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * TLWE1) return;
  const uint64_t g = i / TLWE1;
  const int c = (int)(i - g * TLWE1);
  t[i] += t[(B + g) * TLWE1 + c] + (c == RING_N ? MU : 0u);
}

hipError_t launch_mux_prologue(const uint32_t* sel, const uint32_t* in1, const uint32_t* in0, uint32_t* abar,
                               uint64_t B, hipStream_t st) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mux_prologue, dim3((unsigned)((2 * B * TLWE0 + 255) / 256)), dim3(256), 0, st, sel, in1, in0,
                     abar, B);
  return hipGetLastError();
}

hipError_t launch_mux_combine(uint32_t* t, uint64_t B, hipStream_t st) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mux_combine, dim3((unsigned)((B * TLWE1 + 255) / 256)), dim3(256), 0, st, t, B);
  return hipGetLastError();
}

// ------------------------------------------------------------------ blind rotation
// Raises the dynamic-LDS limit of the kernels that use more than 64 KiB (once, at context
// creation, outside any stream capture).
hipError_t init_kernel_attributes() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_blind_rotate<4>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)br_lds_bytes(4));
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_blind_rotate<8>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)br_lds_bytes(8));
  return e;
}

hipError_t blind_rotate_capacity(int device, uint64_t (&cap)[kBrShapes]) {
  int cus = 0, n4 = 0, n8 = 0, nw = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n4, reinterpret_cast<const void*>(&k_blind_rotate<4>), 256,
                                                     br_lds_bytes(4));
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n8, reinterpret_cast<const void*>(&k_blind_rotate<8>), 512,
                                                     br_lds_bytes(8));
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nw, reinterpret_cast<const void*>(&k_blind_rotate_wide),
                                                     BRW_WAVES * 64, brw_lds_bytes());
  if (e != hipSuccess) return e;
  static_assert(kBrWaveChoices[0] == 4 && kBrWaveChoices[1] == 8 && kBrWaveChoices[2] == 3 && kBrWaveChoices[3] == 32 &&
                    kBrWaveChoices[4] == 33,
                "shape order");
  cap[0] = (uint64_t)(n4 > 0 ? n4 : 1) * (uint64_t)cus * 4;
  cap[1] = (uint64_t)(n8 > 0 ? n8 : 1) * (uint64_t)cus * 8;
  cap[2] = (uint64_t)(nw > 0 ? nw : 1) * (uint64_t)cus;
  // matrix-core form: one workgroup per compute unit holds half a tile of MF_TILE gates
  cap[3] = (uint64_t)cus * MF_TILE / 2;
  // split form: its shortest launch, one tile
  cap[4] = MF_TILE;
  return hipSuccess;
}

hipError_t launch_blind_rotate(const vsp_context* ctx, const uint8_t* ops, const uint32_t* abar, uint32_t* tlwe1,
                               uint32_t* trlwe, uint64_t B, int waves, hipStream_t st, const uint64_t* bkn,
                               const uint64_t* const* keytab, const uint16_t* kid, void* mf_work, bool instrument,
                               const int8_t* const* tile_mfkeys) {
  if (B == 0) return hipSuccess;
  if (bkn == nullptr) bkn = ctx->bkn;
  if (waves <= 0) waves = ctx->tune.br_waves(B);
  if (br_matrix_form(waves)) {
    const bool own = keytab == nullptr && bkn == ctx->bkn && ctx->mf_key != nullptr;
    if (mf_work != nullptr && (own || tile_mfkeys != nullptr))
      return waves == 32 ? launch_blind_rotate_mfma(ctx, ops, abar, tlwe1, trlwe, B, mf_work, st, instrument, tile_mfkeys)
                         : launch_blind_rotate_mfsplit(ctx, ops, abar, tlwe1, trlwe, B, mf_work,
                                                       ctx->tune.split_groups_for(B, ctx->cus), st, instrument,
                                                       tile_mfkeys);
    waves = ctx->tune.br_waves(B, true);
  }
  if (waves == 3) {
    hipLaunchKernelGGL(k_blind_rotate_wide, dim3((unsigned)B), dim3(BRW_WAVES * 64), brw_lds_bytes(), st, bkn,
                       ctx->tw, ops, abar, tlwe1, trlwe, B, keytab, kid);
  } else if (waves == 4) {
    hipLaunchKernelGGL(k_blind_rotate<4>, dim3((unsigned)((B + 3) / 4)), dim3(256), br_lds_bytes(4), st, bkn,
                       ctx->tw, ops, abar, tlwe1, trlwe, B, keytab, kid);
  } else {
    hipLaunchKernelGGL(k_blind_rotate<8>, dim3((unsigned)((B + 7) / 8)), dim3(512), br_lds_bytes(8), st, bkn,
                       ctx->tw, ops, abar, tlwe1, trlwe, B, keytab, kid);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ key switching
// out = (0, b') - sum_{j,p} KSK[j][p][v_{j,p}], v_{j,p} the p-th base-4 digit (most
// significant first) of a'_j rounded to 16 bits. The device key has a zero row at v = 0 so
// the loop is branch-free. One workgroup of 256 threads per gate, 3 coefficients per thread.
__global__ __launch_bounds__(256) void k_keyswitch(const u32* __restrict__ ksk, const uint8_t* __restrict__ ops,
                                                   const u32* __restrict__ tlwe1, const u32* __restrict__ idxo,
                                                   u32* __restrict__ out, uint64_t B) {
  const uint64_t g = blockIdx.x;
  if (g >= B) return;
  if (ops && !op_bootstraps(ops[g])) return;
  const u32* in = tlwe1 + g * TLWE1;
  const int tid = threadIdx.x;
  u32 acc0 = 0, acc1 = 0, acc2 = 0;
  const int c0 = tid, c1 = tid + 256, c2 = tid + 512;
  const bool has2 = c2 < TLWE0;
  for (int j = 0; j < RING_N; j++) {
    const u32 ahat = __builtin_amdgcn_readfirstlane(in[j]) + (1u << 15);
    const u32* base = ksk + (size_t)j * KS_T * 4 * TLWE0;
#pragma unroll
    for (int p = 0; p < KS_T; p++) {
      const u32 v = (ahat >> (30 - 2 * p)) & 3u;
      const u32* row = base + (size_t)(p * 4 + v) * TLWE0;
      acc0 += row[c0];
      acc1 += row[c1];
      if (has2) acc2 += row[c2];
    }
  }
  const uint64_t ro = idxo ? idxo[g] : g;
  u32* o = out + ro * TLWE0;
  const u32 b = in[RING_N];
  o[c0] = 0u - acc0;
  o[c1] = 0u - acc1;
  if (has2) o[c2] = (c2 == LWE_N ? b : 0u) - acc2;
}

// Gate types and output rows of a tile's G gates, loaded together (unconditionally, index
// clamped into the batch: a guarded load becomes a branch after which the compiler waits for
// it, one round trip per gate).
template <int G>
__device__ __forceinline__ void tile_rows(const uint8_t* ops, const u32* idxo, uint64_t g0, int ng, bool (&live)[G],
                                          uint64_t (&ro)[G]) {
  uint8_t opv[G];
  u32 iv[G];
#pragma unroll
  for (int g = 0; g < G; g++) {
    opv[g] = 0;  // a bootstrapping gate type
    iv[g] = 0;
  }
  if (ops) {
#pragma unroll
    for (int g = 0; g < G; g++) opv[g] = ops[g0 + (g < ng ? g : 0)];
  }
  if (idxo) {
#pragma unroll
    for (int g = 0; g < G; g++) iv[g] = idxo[g0 + (g < ng ? g : 0)];
  }
#pragma unroll
  for (int g = 0; g < G; g++) {
    live[g] = g < ng && op_bootstraps(opv[g]);
    ro[g] = idxo ? (uint64_t)iv[g] : g0 + g;
  }
}

// Row-stationary form: a workgroup takes a tile of G gates; for every (j, p) it loads the
// three key rows once (3 coefficients per thread) and applies them to all G gates, whose
// digits are wave-uniform values. The key is then read once per tile instead of once per
// gate.
template <int G>
__global__ __launch_bounds__(256) void k_keyswitch_tiled(const u32* __restrict__ ksk, const uint8_t* __restrict__ ops,
                                                         const u32* __restrict__ tlwe1, const u32* __restrict__ idxo,
                                                         u32* __restrict__ out, uint64_t B) {
  const uint64_t g0 = (uint64_t)blockIdx.x * G;
  const int tid = threadIdx.x;
  const int c0 = tid, c1 = tid + 256, c2 = tid + 512;
  const bool has2 = c2 < TLWE0;
  const int ng = (int)((B - g0) < (uint64_t)G ? (B - g0) : (uint64_t)G);
  u32 acc[G][3];
#pragma unroll
  for (int g = 0; g < G; g++) acc[g][0] = acc[g][1] = acc[g][2] = 0;
  for (int j = 0; j < RING_N; j++) {
    u32 ahat[G];
#pragma unroll
    for (int g = 0; g < G; g++)
      ahat[g] = __builtin_amdgcn_readfirstlane(tlwe1[(g0 + (g < ng ? g : 0)) * TLWE1 + j]) + (1u << 15);
    const u32* base = ksk + (size_t)j * KS_T * 4 * TLWE0;
#pragma unroll 2
    for (int p = 0; p < KS_T; p++) {
      const u32* r = base + (size_t)p * 4 * TLWE0;
      const u32 r10 = r[TLWE0 + c0], r11 = r[TLWE0 + c1], r12 = has2 ? r[TLWE0 + c2] : 0u;
      const u32 r20 = r[2 * TLWE0 + c0], r21 = r[2 * TLWE0 + c1], r22 = has2 ? r[2 * TLWE0 + c2] : 0u;
      const u32 r30 = r[3 * TLWE0 + c0], r31 = r[3 * TLWE0 + c1], r32 = has2 ? r[3 * TLWE0 + c2] : 0u;
#pragma unroll
      for (int g = 0; g < G; g++) {
        const u32 v = (ahat[g] >> (30 - 2 * p)) & 3u;
        acc[g][0] += v == 1 ? r10 : v == 2 ? r20 : v == 3 ? r30 : 0u;
        acc[g][1] += v == 1 ? r11 : v == 2 ? r21 : v == 3 ? r31 : 0u;
        acc[g][2] += v == 1 ? r12 : v == 2 ? r22 : v == 3 ? r32 : 0u;
      }
    }
  }
  bool live[G];
  uint64_t ro[G];
  tile_rows<G>(ops, idxo, g0, ng, live, ro);
#pragma unroll
  for (int g = 0; g < G; g++) {
    const uint64_t gg = g0 + g;
    if (live[g]) {
      u32* o = out + ro[g] * TLWE0;
      o[c0] = 0u - acc[g][0];
      o[c1] = 0u - acc[g][1];
      if (has2) o[c2] = (c2 == LWE_N ? tlwe1[gg * TLWE1 + RING_N] : 0u) - acc[g][2];
    }
  }
}

// Split form: the output rows are first set to (0, ..., 0, b'), then workgroups of G gates
// each take a chunk of the j range, stage the three non-zero key rows of every (j, p)
// through LDS (double-buffered, one barrier per (j, p)), add the row selected by each gate's
// digit from LDS, and subtract their partial sums from the output with atomic adds. Integer
// addition mod 2^32 is associative, so the result does not depend on the order.
__global__ __launch_bounds__(256) void k_keyswitch_init(const uint8_t* __restrict__ ops, const u32* __restrict__ tlwe1,
                                                        const u32* __restrict__ idxo, u32* __restrict__ out,
                                                        uint64_t B) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= B * TLWE0) return;
  const uint64_t g = i / TLWE0;
  const int c = (int)(i - g * TLWE0);
  if (ops && !op_bootstraps(ops[g])) return;
  const uint64_t ro = idxo ? idxo[g] : g;
  out[ro * TLWE0 + c] = (c == LWE_N) ? tlwe1[g * TLWE1 + RING_N] : 0u;
}

constexpr int KS_ROW = 640;  // LDS row pitch (u32) of a staged key row

template <int G>
__global__ __launch_bounds__(256) void k_keyswitch_split(const u32* __restrict__ ksk, const uint8_t* __restrict__ ops,
                                                         const u32* __restrict__ tlwe1, const u32* __restrict__ idxo,
                                                         u32* __restrict__ out, uint64_t B, int jchunk) {
  __shared__ u32 rows[2][4 * KS_ROW];  // per buffer: row 0 zero, rows 1..3 the key rows of one (j, p)
  const uint64_t g0 = (uint64_t)blockIdx.x * G;
  const int ng = (int)((B - g0) < (uint64_t)G ? (B - g0) : (uint64_t)G);
  const int j0 = blockIdx.y * jchunk;
  const int j1 = (j0 + jchunk < RING_N) ? j0 + jchunk : RING_N;
  const int tid = threadIdx.x;
  for (int i = tid; i < KS_ROW; i += 256) rows[0][i] = rows[1][i] = 0u;
  constexpr int STAGE = 3 * TLWE0;              // words staged per (j, p)
  constexpr int PER_T = (STAGE + 255) / 256;    // loads per thread
  auto fetch = [&](int j, int p, u32 (&r)[PER_T]) {
    const u32* src = ksk + ((size_t)j * KS_T + p) * 4 * TLWE0 + TLWE0;  // rows v = 1..3 are contiguous
#pragma unroll
    for (int q = 0; q < PER_T; q++) {
      const int i = tid + 256 * q;
      r[q] = (i < STAGE) ? src[i] : 0u;
    }
  };
  auto store = [&](int buf, const u32 (&r)[PER_T]) {
#pragma unroll
    for (int q = 0; q < PER_T; q++) {
      const int i = tid + 256 * q;
      if (i < STAGE) {
        const int v = i / TLWE0;
        rows[buf][(v + 1) * KS_ROW + (i - v * TLWE0)] = r[q];
      }
    }
  };
  u32 acc[G][3];
#pragma unroll
  for (int g = 0; g < G; g++) acc[g][0] = acc[g][1] = acc[g][2] = 0u;
  const int c0 = tid, c1 = tid + 256, c2 = tid + 512;  // c2 valid below TLWE0
  u32 pre[PER_T];
  fetch(j0, 0, pre);
  store(0, pre);
  __syncthreads();
  int buf = 0;
  for (int j = j0; j < j1; j++) {
    u32 ahat[G];
#pragma unroll
    for (int g = 0; g < G; g++) ahat[g] = tlwe1[(g0 + (g < ng ? g : 0)) * TLWE1 + j] + (1u << 15);  // unconditional
#pragma unroll 1
    for (int p = 0; p < KS_T; p++) {
      const bool more = (p + 1 < KS_T) || (j + 1 < j1);
      if (more) fetch(p + 1 < KS_T ? j : j + 1, (p + 1) & (KS_T - 1), pre);
      const u32* rb = rows[buf];
#pragma unroll
      for (int g = 0; g < G; g++) {
        const u32 v = (ahat[g] >> (30 - 2 * p)) & 3u;
        const u32* row = rb + v * KS_ROW;
        acc[g][0] += row[c0];
        acc[g][1] += row[c1];
        if (c2 < TLWE0) acc[g][2] += row[c2];
      }
      if (more) store(buf ^ 1, pre);
      __syncthreads();
      buf ^= 1;
    }
  }
  bool live[G];
  uint64_t ro[G];
  tile_rows<G>(ops, idxo, g0, ng, live, ro);
#pragma unroll
  for (int g = 0; g < G; g++) {
    if (live[g]) {
      u32* o = out + ro[g] * TLWE0;
      __hip_atomic_fetch_add(&o[c0], 0u - acc[g][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&o[c1], 0u - acc[g][1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (c2 < TLWE0) __hip_atomic_fetch_add(&o[c2], 0u - acc[g][2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

hipError_t launch_keyswitch(const vsp_context* ctx, const uint8_t* ops, const uint32_t* tlwe1, const uint32_t* idxo,
                            uint32_t* out, uint64_t B, hipStream_t st, int form, const uint32_t* ksk,
                            const int8_t* ks_mf) {
  if (B == 0) return hipSuccess;
  if (ksk == nullptr) ksk = ctx->ksk;
  if (form < 0) form = ctx->tune.ks_form_for(B);
  if (form == 3) {
    if (ksk == ctx->ksk && ctx->ks_mf != nullptr) return launch_keyswitch_mfma(ctx->ks_mf, ops, tlwe1, idxo, out, B, st);
    if (ksk != ctx->ksk && ks_mf != nullptr) return launch_keyswitch_mfma(ks_mf, ops, tlwe1, idxo, out, B, st);
    form = 2;
  }
  if (form == 2) {
    constexpr int G = 16;
    const uint64_t tiles = (B + G - 1) / G;
    // split the j range so that the launch has about 2048 workgroups (chunks of >= 16 j)
    uint64_t split = 2048 / tiles;
    split = split < 1 ? 1 : (split > RING_N / 16 ? RING_N / 16 : split);
    const int jchunk = (int)((RING_N + split - 1) / split);
    const unsigned ychunks = (unsigned)((RING_N + jchunk - 1) / jchunk);
    hipLaunchKernelGGL(k_keyswitch_init, dim3((unsigned)((B * TLWE0 + 255) / 256)), dim3(256), 0, st, ops, tlwe1, idxo,
                       out, B);
    hipLaunchKernelGGL(k_keyswitch_split<G>, dim3((unsigned)tiles, ychunks), dim3(256), 0, st, ksk, ops, tlwe1,
                       idxo, out, B, jchunk);
  } else if (form == 1) {
    constexpr int G = 16;
    hipLaunchKernelGGL(k_keyswitch_tiled<G>, dim3((unsigned)((B + G - 1) / G)), dim3(256), 0, st, ksk, ops, tlwe1,
                       idxo, out, B);
  } else {
    hipLaunchKernelGGL(k_keyswitch, dim3((unsigned)B), dim3(256), 0, st, ksk, ops, tlwe1, idxo, out, B);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ test kernels
__global__ __launch_bounds__(256) void k_ext_product(const u64* __restrict__ Cn, const u32* __restrict__ x,
                                                     u32* __restrict__ out, const u64* __restrict__ tw, uint64_t J) {
  __shared__ u32 lds[4 * WAVE_T_U32];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t j = (uint64_t)blockIdx.x * 4 + wave;
  if (j >= J) return;
  const int lane = threadIdx.x & 63, l = lane & 31, h = lane >> 5;
  u32* reg = lds + wave * WAVE_T_U32 + h * TREGION;
  const u32* xp = x + j * 2 * RING_N + h * RING_N;
  u32 D[32], acc[32];
#pragma unroll
  for (int t = 0; t < 32; t++) D[t] = xp[l + 32 * t];
  external_product(OperandDigits{D}, Cn + j * TRGSW_NTT_U64, tw, tw + 1024, reg, lane, acc);
  u32* o = out + j * 2 * RING_N + h * RING_N;
#pragma unroll
  for (int t = 0; t < 32; t++) o[l + 32 * t] = acc[t];
}

hipError_t launch_ext_product(const vsp_context* ctx, const uint64_t* Cn, const uint32_t* x, uint32_t* out, uint64_t J,
                              hipStream_t st) {
  if (J == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ext_product, dim3((unsigned)((J + 3) / 4)), dim3(256), 0, st, Cn, x, out, ctx->tw, J);
  return hipGetLastError();
}

// Negacyclic product through the NTT: lanes 0-31 transform a, lanes 32-63 transform b,
// the pointwise product is formed in lanes 0-31 and transformed back there.
__global__ __launch_bounds__(256) void k_polymul(const int32_t* __restrict__ a, const u32* __restrict__ b,
                                                 u32* __restrict__ out, const u64* __restrict__ tw, u64 ninv,
                                                 uint64_t J) {
  __shared__ u32 lds[4 * WAVE_T_U32];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t j = (uint64_t)blockIdx.x * 4 + wave;
  if (j >= J) return;
  const int lane = threadIdx.x & 63, l = lane & 31, h = lane >> 5;
  u32* reg = lds + wave * WAVE_T_U32 + h * TREGION;
  u64 v[32];
#pragma unroll
  for (int t = 0; t < 32; t++)
    v[t] = h ? (u64)b[j * RING_N + l + 32 * t] : gl_from_i32(a[j * RING_N + l + 32 * t]);
  ntt_forward(v, tw, reg, l);
#pragma unroll
  for (int s = 0; s < 32; s++) {
    const u64 other = __shfl_xor(v[s], 32);
    v[s] = gl_mul(gl_mul(v[s], other), ninv);
  }
  u32 z[32];
  ntt_inverse_lift(v, tw + 1024, reg, l, z);
  if (h == 0) {
#pragma unroll
    for (int t = 0; t < 32; t++) out[j * RING_N + l + 32 * t] = z[t];
  }
}

hipError_t launch_polymul(const vsp_context* ctx, const int32_t* a, const uint32_t* b, uint32_t* out, uint64_t J,
                          hipStream_t st) {
  if (J == 0) return hipSuccess;
  const u64 ninv = gl_powmod_const(RING_N, GL_P - 2);
  hipLaunchKernelGGL(k_polymul, dim3((unsigned)((J + 3) / 4)), dim3(256), 0, st, a, b, out, ctx->tw, ninv, J);
  return hipGetLastError();
}

}  // namespace vsp
