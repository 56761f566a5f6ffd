// CMUX Memory (Sec. 8): ROM reads by a packed LUT (CMUX tree + rotation CMUXes), RAM reads
// by per-bit CMUX trees, and the RAM write (read unit, control unit, write bars, refresh).

#include "vsp_internal.h"

namespace vsp {

constexpr int TRLWE_WORDS = 2 * RING_N;
constexpr int TRGSW_WORDS = 2 * GADGET_L * 2 * RING_N;

// ------------------------------------------------------------------ kernels
// The CMUX kernels run one CMUX chain per wave, WAVES waves per workgroup. The workgroup's
// LDS holds the twiddle tables, then per wave a polynomial pair (2N u32: lanes 0-31 own the
// a polynomial, lanes 32-63 the b polynomial, coefficient l + 32 t in lane l) and the wave's
// two transpose regions. Keeping the pair in LDS instead of registers and reading the
// gadget digits from it in every round leaves the external product within 256 VGPRs, so a
// SIMD runs two waves.
constexpr int MEM_WAVE_U32 = 2 * RING_N + WAVE_T_U32;
constexpr size_t mem_lds_bytes(int waves) { return 2048 * 8 + (size_t)waves * MEM_WAVE_U32 * 4; }

template <int WAVES>
__device__ __forceinline__ void stage_twiddles(u64* tws, const u64* __restrict__ tw) {
  for (int i = threadIdx.x; i < 2048; i += WAVES * 64) tws[i] = tw[i];
  __syncthreads();
}

// z = C (ext) P for the pair P at the start of this wave's LDS area; the wave's transpose
// regions follow the pair. The product of external_product, with the digits re-read from LDS
// and every LDS and key address formed anew in each round (from an opaque copy of the lane
// index), so that none of them stays live across the rounds. KEY_LATE issues a round's first
// key loads after its forward transform instead of before its digits: fewer live registers
// during the transform, less latency hidden (the choice that keeps each caller's register
// spills smallest at 256 VGPRs).
template <bool KEY_LATE>
__device__ __forceinline__ void ext_product_lds(u32* wbase, const u64* __restrict__ C, const u64* tws, int lane,
                                                u32 (&z)[32]) {
  u64 sum[32];
#pragma unroll
  for (int s = 0; s < 32; s++) sum[s] = 0;
#pragma unroll 1
  for (int k = 0; k < GADGET_L; k++) {
    const int ln = opaque_lane(lane);
    const int li = ln & 31;
    const u32* p = wbase + (ln >> 5) * RING_N + li;
    const ulonglong2* key = reinterpret_cast<const ulonglong2*>(C) + (size_t)k * 32 * 64 + ln;
    ulonglong2 kc[KCH];
    if (!KEY_LATE) {
#pragma unroll
      for (int q = 0; q < KCH; q++) kc[q] = key[q * 64];
    }
    u64 x[32];
    const int sh = 32 - BG_BIT * (k + 1);
#pragma unroll
    for (int t = 0; t < 32; t++) x[t] = gadget_digit(p[32 * t], sh);
    ntt_forward<true>(x, tws, wbase + 2 * RING_N + (ln >> 5) * TREGION, li);
    if (KEY_LATE) {
#pragma unroll
      for (int q = 0; q < KCH; q++) kc[q] = key[q * 64];
    }
#pragma unroll
    for (int c = 0; c < 32 / KCH; c++) {
      ulonglong2 kn[KCH];
      if (c + 1 < 32 / KCH) {
#pragma unroll
        for (int q = 0; q < KCH; q++) kn[q] = key[(KCH * (c + 1) + q) * 64];
      }
#pragma unroll
      for (int q = 0; q < KCH; q++) {
        const int s = KCH * c + q;
        u64 xa, xb;
        both_halves(x[s], xa, xb);
        sum[s] = gl_add(sum[s], gl_dot2(xa, kc[q].x, xb, kc[q].y));
      }
      __builtin_amdgcn_sched_barrier(0);
      if (c + 1 < 32 / KCH) {
#pragma unroll
        for (int q = 0; q < KCH; q++) kc[q] = kn[q];
      }
    }
  }
  const int ln = opaque_lane(lane);
  ntt_inverse_lift(sum, tws + 1024, wbase + 2 * RING_N + (ln >> 5) * TREGION, ln & 31, z);
}

// One wave per CMUX: out = x0 + C (ext) (x1 - x0).
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_cmux_tree_level(const u64* __restrict__ sel, uint64_t sel_r_stride,
                                                                int selbit, const u32* __restrict__ in, uint64_t s_r,
                                                                uint64_t s_b, u32* __restrict__ out, uint64_t R,
                                                                uint64_t nb, uint64_t half,
                                                                const u64* __restrict__ tw) {
  extern __shared__ u64 lds[];
  stage_twiddles<WAVES>(lds, tw);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t job = (uint64_t)blockIdx.x * WAVES + wave;
  if (job >= R * nb * half) return;
  const int lane = threadIdx.x & 63, l = lane & 31, h = lane >> 5;
  const uint64_t m = job % half, rb = job / half, blk = rb % nb, r = rb / nb;
  const u32* x0 = in + r * s_r + blk * s_b + (2 * m) * TRLWE_WORDS + h * RING_N;
  const u32* x1 = x0 + TRLWE_WORDS;
  u32* wbase = reinterpret_cast<u32*>(lds + 2048) + wave * MEM_WAVE_U32;
  u32* buf = wbase + h * RING_N;
#pragma unroll
  for (int t = 0; t < 32; t++) buf[l + 32 * t] = x1[l + 32 * t] - x0[l + 32 * t];
  wave_lds_sync();
  u32 z[32];
  ext_product_lds<false>(wbase, sel + (r * sel_r_stride + (uint64_t)selbit) * TRGSW_NTT_U64, lds, lane, z);
  // the epilogue's addresses are formed anew here rather than kept live across the product
  const int ln = opaque_lane(lane);
  const u32* y0 = in + r * s_r + blk * s_b + (2 * m) * TRLWE_WORDS + (ln >> 5) * RING_N + (ln & 31);
  u32* o = out + job * TRLWE_WORDS + (ln >> 5) * RING_N + (ln & 31);
#pragma unroll
  for (int t = 0; t < 32; t++) o[32 * t] = y0[32 * t] + z[t];
}

// One wave per read: R <- CMUX(C_j, R, X^{-w 2^j} R) = R + C_j (ext) (X^{-w 2^j} R - R), j
// ascending. R lives in the wave's LDS buffer; the digits of the rotation difference are
// formed from it in every round, and the product is added to it in place.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_rom_rotate(const u64* __restrict__ sel, uint64_t sel_r_stride,
                                                           u32* __restrict__ accbuf, uint64_t R, int rotbits, int w,
                                                           const u64* __restrict__ tw) {
  extern __shared__ u64 lds[];
  stage_twiddles<WAVES>(lds, tw);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t r = (uint64_t)blockIdx.x * WAVES + wave;
  if (r >= R) return;
  const int lane = threadIdx.x & 63, l = lane & 31, h = lane >> 5;
  u32* wbase = reinterpret_cast<u32*>(lds + 2048) + wave * MEM_WAVE_U32;
  u32* p = accbuf + r * TRLWE_WORDS + h * RING_N;
  {
    u32* accs = wbase + h * RING_N;
#pragma unroll
    for (int t = 0; t < 32; t++) accs[l + 32 * t] = p[l + 32 * t];
  }
  wave_lds_sync();
  for (int j = 0; j < rotbits; j++) {
    const int k = (2 * RING_N - (w << j)) & (2 * RING_N - 1);
    const int ln = opaque_lane(lane);
    const int li = ln & 31, hi = ln >> 5;
    u32* accs = wbase + hi * RING_N;
    auto digits = [&](int sh, u64 (&x)[32]) {
#pragma unroll
      for (int t = 0; t < 32; t++) {
        const int idx = (li + 32 * t - k) & (2 * RING_N - 1);
        u32 v = accs[idx & (RING_N - 1)];
        if (idx & RING_N) v = 0u - v;
        x[t] = gadget_digit(v - accs[li + 32 * t], sh);
      }
    };
    u32 z[32];
    external_product(digits, sel + (r * sel_r_stride + (uint64_t)j) * TRGSW_NTT_U64, lds, lds + 1024,
                     wbase + 2 * RING_N + hi * TREGION, ln, z);
#pragma unroll
    for (int t = 0; t < 32; t++)
      __hip_atomic_fetch_add(&accs[li + 32 * t], z[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    wave_lds_sync();
  }
  const u32* accs = wbase + h * RING_N;
#pragma unroll
  for (int t = 0; t < 32; t++) p[l + 32 * t] = accs[l + 32 * t];
}

// SampleExtract_h for h < W: out[r][h] (N + 1 words) from in[r] = (A, B).
__global__ __launch_bounds__(256) void k_sample_extract(const u32* __restrict__ in, u32* __restrict__ out, uint64_t R,
                                                        int W) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t per = (uint64_t)W * (RING_N + 1);
  if (i >= R * per) return;
  const uint64_t r = i / per;
  const int rem = (int)(i - r * per), hh = rem / (RING_N + 1), j = rem - hh * (RING_N + 1);
  const u32* c = in + r * TRLWE_WORDS;
  u32 v;
  if (j == RING_N) v = c[RING_N + hh];
  else if (j <= hh) v = c[hh - j];
  else v = 0u - c[RING_N + hh - j];
  out[i] = v;
}

// Control unit output u_i = acc[i] + acc[w + i] + (0, mu X^0).
__global__ __launch_bounds__(256) void k_ram_control(const u32* __restrict__ acc2, u32* __restrict__ u, int w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= w * TRLWE_WORDS) return;
  const int bit = i / TRLWE_WORDS, c = i - bit * TRLWE_WORDS;
  u[i] = acc2[i] + acc2[(size_t)(w + bit) * TRLWE_WORDS + c] + (c == RING_N ? MU : 0u);
}

// One wave per write bar (bit i, address A): y = u_i; for d < v: y = CMUX(s_d, R[i][A], y)
// = R[i][A] + s_d (ext) (y - R[i][A]) with s_d = C_d (bit d of A is 1) or G - C_d (0);
// then SampleExtract_0(y) into tlwe1[i 2^v + A]. The chain runs on the difference
// D = y - R[i][A]: D starts as u_i - R[i][A], each step replaces it by s_d (ext) D, and the
// result is y = R[i][A] + D. D lives in the wave's LDS buffer.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_ram_bars(const u64* __restrict__ sel, const u64* __restrict__ selneg,
                                                         const u32* __restrict__ ram, const u32* __restrict__ u,
                                                         u32* __restrict__ tlwe1, int v, int w,
                                                         const u64* __restrict__ tw) {
  extern __shared__ u64 lds[];
  stage_twiddles<WAVES>(lds, tw);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t bar = (uint64_t)blockIdx.x * WAVES + wave;
  if (bar >= ((uint64_t)w << v)) return;
  const int lane = threadIdx.x & 63, l = lane & 31, h = lane >> 5;
  const uint64_t i = bar >> v, A = bar & ((1ull << v) - 1);
  u32* wbase = reinterpret_cast<u32*>(lds + 2048) + wave * MEM_WAVE_U32;
  u32* buf = wbase + h * RING_N;
  const u32* old = ram + bar * TRLWE_WORDS + h * RING_N;
  const u32* ui = u + i * TRLWE_WORDS + h * RING_N;
#pragma unroll
  for (int t = 0; t < 32; t++) buf[l + 32 * t] = ui[l + 32 * t] - old[l + 32 * t];
  wave_lds_sync();
  for (int d = 0; d < v; d++) {
    const u64* C = (((A >> d) & 1) ? sel : selneg) + (size_t)d * TRGSW_NTT_U64;
    u32 z[32];
    ext_product_lds<true>(wbase, C, lds, lane, z);
    // a lane reads and writes only its own coefficients of D
#pragma unroll
    for (int t = 0; t < 32; t++) buf[l + 32 * t] = z[t];
    wave_lds_sync();
  }
  const int ln = opaque_lane(lane);  // addresses formed anew, not kept live across the chain
  const int li = ln & 31;
  const u32* cell = ram + bar * TRLWE_WORDS + (ln >> 5) * RING_N;
  const u32* dfin = wbase + (ln >> 5) * RING_N;
  u32 y[32];
#pragma unroll
  for (int t = 0; t < 32; t++) y[t] = cell[li + 32 * t] + dfin[li + 32 * t];
  u32* out = tlwe1 + bar * (RING_N + 1);
  if (h == 0) {
#pragma unroll
    for (int t = 0; t < 32; t++) {
      const int j = l + 32 * t;
      out[(RING_N - j) & (RING_N - 1)] = (j == 0) ? y[t] : 0u - y[t];
    }
  } else if (l == 0) {
    out[RING_N] = y[0];
  }
}

// G - C: negate every coefficient of C and add the gadget constants of the trivial TRGSW(1).
__global__ __launch_bounds__(256) void k_gadget_minus(const u32* __restrict__ C, u32* __restrict__ out, uint64_t count) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count * TRGSW_WORDS) return;
  const int within = (int)(i % TRGSW_WORDS);
  const int row = within / TRLWE_WORDS, rem = within % TRLWE_WORDS, col = rem / RING_N, coef = rem % RING_N;
  u32 g = 0;
  if (coef == 0) {
    if (row < GADGET_L && col == 0) g = 1u << (32 - BG_BIT * (row + 1));
    if (row >= GADGET_L && col == 1) g = 1u << (32 - BG_BIT * (row - GADGET_L + 1));
  }
  out[i] = g - C[i];
}

// Broadcast one TRLWE to R slots.
__global__ __launch_bounds__(256) void k_broadcast(const u32* __restrict__ src, u32* __restrict__ dst, uint64_t R) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * TRLWE_WORDS) return;
  dst[i] = src[i % TRLWE_WORDS];
}

// ------------------------------------------------------------------ launchers
static unsigned blocks_for(uint64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// The CMUX kernels in two shapes: eight waves per workgroup (two waves per SIMD once every CU
// holds one workgroup) for wide launches, one wave per workgroup for narrow ones, where
// spreading the few chains over all CUs shortens the launch.
hipError_t init_memory_kernel_attributes() {
  const void* fns[] = {reinterpret_cast<const void*>(&k_cmux_tree_level<8>),
                       reinterpret_cast<const void*>(&k_rom_rotate<8>),
                       reinterpret_cast<const void*>(&k_ram_bars<8>),
                       reinterpret_cast<const void*>(&k_cmux_tree_level<1>),
                       reinterpret_cast<const void*>(&k_rom_rotate<1>),
                       reinterpret_cast<const void*>(&k_ram_bars<1>)};
  for (int f = 0; f < 6; f++) {
    const hipError_t e =
        hipFuncSetAttribute(fns[f], hipFuncAttributeMaxDynamicSharedMemorySize, (int)mem_lds_bytes(f < 3 ? 8 : 1));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static bool wide_launch(const vsp_context* ctx, uint64_t chains) { return chains >= 8ull * (uint64_t)ctx->cus; }

hipError_t launch_cmux_tree_level(const vsp_context* ctx, const uint64_t* sel, uint64_t sel_r_stride, int selbit,
                                  const uint32_t* in, uint64_t s_r, uint64_t s_b, uint32_t* out, uint64_t R,
                                  uint64_t nb, uint64_t W, hipStream_t st) {
  const uint64_t jobs = R * nb * (W / 2);
  if (jobs == 0) return hipSuccess;
  if (wide_launch(ctx, jobs))
    hipLaunchKernelGGL(k_cmux_tree_level<8>, dim3(blocks_for(jobs, 8)), dim3(512), mem_lds_bytes(8), st, sel,
                       sel_r_stride, selbit, in, s_r, s_b, out, R, nb, W / 2, ctx->tw);
  else
    hipLaunchKernelGGL(k_cmux_tree_level<1>, dim3(blocks_for(jobs, 1)), dim3(64), mem_lds_bytes(1), st, sel,
                       sel_r_stride, selbit, in, s_r, s_b, out, R, nb, W / 2, ctx->tw);
  return hipGetLastError();
}

hipError_t launch_rom_rotate(const vsp_context* ctx, const uint64_t* sel, uint64_t sel_r_stride, uint32_t* acc,
                             uint64_t R, int rotbits, int w, hipStream_t st) {
  if (R == 0 || rotbits == 0) return hipSuccess;
  if (wide_launch(ctx, R))
    hipLaunchKernelGGL(k_rom_rotate<8>, dim3(blocks_for(R, 8)), dim3(512), mem_lds_bytes(8), st, sel, sel_r_stride,
                       acc, R, rotbits, w, ctx->tw);
  else
    hipLaunchKernelGGL(k_rom_rotate<1>, dim3(blocks_for(R, 1)), dim3(64), mem_lds_bytes(1), st, sel, sel_r_stride,
                       acc, R, rotbits, w, ctx->tw);
  return hipGetLastError();
}

hipError_t launch_sample_extract(const uint32_t* in, uint32_t* out, uint64_t R, int W, hipStream_t st) {
  const uint64_t n = R * (uint64_t)W * (RING_N + 1);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample_extract, dim3(blocks_for(n, 256)), dim3(256), 0, st, in, out, R, W);
  return hipGetLastError();
}

hipError_t launch_ram_control(const uint32_t* acc2, uint32_t* u, int w, hipStream_t st) {
  hipLaunchKernelGGL(k_ram_control, dim3(blocks_for((uint64_t)w * TRLWE_WORDS, 256)), dim3(256), 0, st, acc2, u, w);
  return hipGetLastError();
}

hipError_t launch_ram_bars(const vsp_context* ctx, const uint64_t* sel, const uint64_t* selneg, const uint32_t* ram,
                           const uint32_t* u, uint32_t* tlwe1, int v, int w, hipStream_t st) {
  const uint64_t bars = (uint64_t)w << v;
  if (wide_launch(ctx, bars))
    hipLaunchKernelGGL(k_ram_bars<8>, dim3(blocks_for(bars, 8)), dim3(512), mem_lds_bytes(8), st, sel, selneg, ram, u,
                       tlwe1, v, w, ctx->tw);
  else
    hipLaunchKernelGGL(k_ram_bars<1>, dim3(blocks_for(bars, 1)), dim3(64), mem_lds_bytes(1), st, sel, selneg, ram, u,
                       tlwe1, v, w, ctx->tw);
  return hipGetLastError();
}

hipError_t launch_gadget_minus(const uint32_t* C, uint32_t* out, uint64_t count, hipStream_t st) {
  const uint64_t n = count * TRGSW_WORDS;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gadget_minus, dim3(blocks_for(n, 256)), dim3(256), 0, st, C, out, count);
  return hipGetLastError();
}

static hipError_t launch_broadcast(const uint32_t* src, uint32_t* dst, uint64_t R, hipStream_t st) {
  hipLaunchKernelGGL(k_broadcast, dim3(blocks_for(R * TRLWE_WORDS, 256)), dim3(256), 0, st, src, dst, R);
  return hipGetLastError();
}

static int ilog2(uint64_t x) {
  int r = 0;
  while ((1ull << r) < x) r++;
  return r;
}

// CMUX trees of `levels` levels over `nb` blocks per read (cells [nb][2^levels] shared by all
// reads, block stride s_b words), address bits `bit0`.. of each read's selectors. Leaves
// the R * nb results in *result (one of two ping-pong buffers a, b).
static hipError_t run_trees(const vsp_context* ctx, const uint64_t* sel, uint64_t sel_r_stride, int bit0, int levels,
                            const uint32_t* cells, uint64_t s_b, uint64_t R, uint64_t nb, uint32_t* a, uint32_t* b,
                            uint32_t** result, hipStream_t st) {
  uint64_t W = 1ull << levels;
  const uint32_t* in = cells;
  uint64_t s_r = 0, sb = s_b;
  uint32_t* bufs[2] = {a, b};
  int cur = 0;
  for (int d = 0; d < levels; d++) {
    uint32_t* out = bufs[cur];
    hipError_t e = launch_cmux_tree_level(ctx, sel, sel_r_stride, bit0 + d, in, s_r, sb, out, R, nb, W, st);
    if (e != hipSuccess) return e;
    W /= 2;
    in = out;
    sb = W * TRLWE_WORDS;
    s_r = nb * sb;
    cur ^= 1;
  }
  if (levels == 0) {
    // a single cell (ROM with one polynomial): give every read its own copy
    hipError_t e = launch_broadcast(cells, a, R, st);
    if (e != hipSuccess) return e;
    *result = a;
    return hipSuccess;
  }
  *result = const_cast<uint32_t*>(in);
  return hipSuccess;
}

// Input-wire and opcode tables of the control unit's 2w gates over the rows
// src = [f, x_0 .. x_{w-1}, r_0 .. r_{w-1}]: gate i < w is AND(f, x_i), gate w + i is
// ANDNOT(r_i, f) (idx0 = idx[0, 2w), idx1 = idx[2w, 4w)). Written on the device so that the
// write stays asynchronous.
__global__ void k_ram_control_tables(uint32_t* __restrict__ idx, uint8_t* __restrict__ ops, uint32_t w) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= w) return;
  idx[i] = 0;
  idx[2 * w + i] = 1 + i;
  idx[w + i] = 1 + w + i;
  idx[3 * w + i] = 0;
  ops[i] = VSP_AND;
  ops[w + i] = VSP_ANDNOT;
}

static hipError_t launch_ram_control_tables(uint32_t* idx, uint8_t* ops, uint32_t w, hipStream_t st) {
  hipLaunchKernelGGL(k_ram_control_tables, dim3((w + 255) / 256), dim3(256), 0, st, idx, ops, w);
  return hipGetLastError();
}

}  // namespace vsp

using namespace vsp;

extern "C" {

vsp_status vsp_rom_read(vsp_context* ctx, const uint32_t* d_rom, uint32_t P, const uint32_t* d_addr, uint32_t v,
                        uint32_t w, uint32_t* d_out, uint64_t R, void* stream) {
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  if (R == 0) return VSP_OK;
  if (w == 0 || (w & (w - 1)) || w > (uint32_t)RING_N) return fail(VSP_E_ARG, "w must be a power of two <= N");
  const int rotbits = ilog2(RING_N / w);
  if (v < (uint32_t)rotbits || v > 32) return fail(VSP_E_ARG, "v must be at least log2(N / w)");
  if ((uint64_t)P != (1ull << (v - rotbits))) return fail(VSP_E_ARG, "P must equal 2^(v - log2(N / w))");
  if (R > (1ull << 24) || R * w > kMaxLaunch) return fail(VSP_E_ARG, "R too large (R * w must not exceed 2^22)");
  VSP_HIP(hipSetDevice(ctx->device));
  vsp_status s;
  const size_t rom_b = (size_t)P * TRLWE_WORDS * 4, addr_b = (size_t)R * v * TRGSW_WORDS * 4,
               out_b = (size_t)R * w * (LWE_N + 1) * 4;
  if ((s = check_device_range(ctx, d_rom, rom_b, "d_rom"))) return s;
  if ((s = check_device_range(ctx, d_addr, addr_b, "d_addr"))) return s;
  if ((s = check_device_range(ctx, d_out, out_b, "d_out"))) return s;
  if ((s = check_no_overlap(d_out, out_b, d_rom, rom_b, "d_out and d_rom"))) return s;
  if ((s = check_no_overlap(d_out, out_b, d_addr, addr_b, "d_out and d_addr"))) return s;
  const uint64_t half = P > 1 ? P / 2 : 1;
  if ((s = scratch_reserve(ctx, ctx->ntt_sel, (size_t)R * v * TRGSW_NTT_U64 * 8))) return s;
  if ((s = scratch_reserve(ctx, ctx->mem_a, (size_t)R * half * TRLWE_WORDS * 4))) return s;
  if ((s = scratch_reserve(ctx, ctx->mem_b, (size_t)R * half * TRLWE_WORDS * 4))) return s;
  if ((s = scratch_reserve(ctx, ctx->tlwe1, (size_t)R * w * (RING_N + 1) * 4))) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint64_t* sel = static_cast<uint64_t*>(ctx->ntt_sel.ptr);
  hipError_t e;
  if ((e = launch_trgsw_to_ntt(ctx, d_addr, sel, R * v, st)) != hipSuccess) return hip_fail(e, "selector conversion");
  uint32_t* acc = nullptr;
  if ((e = run_trees(ctx, sel, v, rotbits, (int)(v - rotbits), d_rom, 0, R, 1, static_cast<uint32_t*>(ctx->mem_a.ptr),
                     static_cast<uint32_t*>(ctx->mem_b.ptr), &acc, st)) != hipSuccess)
    return hip_fail(e, "ROM tree");
  if ((e = launch_rom_rotate(ctx, sel, v, acc, R, rotbits, (int)w, st)) != hipSuccess) return hip_fail(e, "ROM rotate");
  uint32_t* t1 = static_cast<uint32_t*>(ctx->tlwe1.ptr);
  if ((e = launch_sample_extract(acc, t1, R, (int)w, st)) != hipSuccess) return hip_fail(e, "sample extract");
  if ((e = launch_keyswitch(ctx, nullptr, t1, nullptr, d_out, R * w, st)) != hipSuccess) return hip_fail(e, "key switch");
  return VSP_OK;
}

vsp_status vsp_ram_read(vsp_context* ctx, const uint32_t* d_ram, uint32_t v, uint32_t w, const uint32_t* d_addr,
                        uint32_t* d_out, uint64_t R, void* stream) {
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  if (R == 0) return VSP_OK;
  if (v < 1 || v > 16) return fail(VSP_E_ARG, "v must be in [1, 16]");
  if (w < 1 || w > 1024) return fail(VSP_E_ARG, "w must be in [1, 1024]");
  if (R > (1ull << 20) || R * w > kMaxLaunch) return fail(VSP_E_ARG, "R too large (R * w must not exceed 2^22)");
  VSP_HIP(hipSetDevice(ctx->device));
  vsp_status s;
  const uint64_t cells = (uint64_t)w << v;
  const size_t ram_b = cells * TRLWE_WORDS * 4, addr_b = (size_t)R * v * TRGSW_WORDS * 4,
               out_b = (size_t)R * w * (LWE_N + 1) * 4;
  if ((s = check_device_range(ctx, d_ram, ram_b, "d_ram"))) return s;
  if ((s = check_device_range(ctx, d_addr, addr_b, "d_addr"))) return s;
  if ((s = check_device_range(ctx, d_out, out_b, "d_out"))) return s;
  if ((s = check_no_overlap(d_out, out_b, d_ram, ram_b, "d_out and d_ram"))) return s;
  if ((s = check_no_overlap(d_out, out_b, d_addr, addr_b, "d_out and d_addr"))) return s;
  if ((s = scratch_reserve(ctx, ctx->ntt_sel, (size_t)R * v * TRGSW_NTT_U64 * 8))) return s;
  const size_t level_b = (size_t)R * (cells / 2) * TRLWE_WORDS * 4;
  if ((s = scratch_reserve(ctx, ctx->mem_a, level_b))) return s;
  if ((s = scratch_reserve(ctx, ctx->mem_b, level_b))) return s;
  if ((s = scratch_reserve(ctx, ctx->tlwe1, (size_t)R * w * (RING_N + 1) * 4))) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint64_t* sel = static_cast<uint64_t*>(ctx->ntt_sel.ptr);
  hipError_t e;
  if ((e = launch_trgsw_to_ntt(ctx, d_addr, sel, R * v, st)) != hipSuccess) return hip_fail(e, "selector conversion");
  uint32_t* res = nullptr;
  if ((e = run_trees(ctx, sel, v, 0, (int)v, d_ram, (1ull << v) * TRLWE_WORDS, R, w, static_cast<uint32_t*>(ctx->mem_a.ptr),
                     static_cast<uint32_t*>(ctx->mem_b.ptr), &res, st)) != hipSuccess)
    return hip_fail(e, "RAM tree");
  uint32_t* t1 = static_cast<uint32_t*>(ctx->tlwe1.ptr);
  if ((e = launch_sample_extract(res, t1, R * w, 1, st)) != hipSuccess) return hip_fail(e, "sample extract");
  if ((e = launch_keyswitch(ctx, nullptr, t1, nullptr, d_out, R * w, st)) != hipSuccess) return hip_fail(e, "key switch");
  return VSP_OK;
}

vsp_status vsp_ram_write(vsp_context* ctx, uint32_t* d_ram, uint32_t v, uint32_t w, const uint32_t* d_addr,
                         const uint32_t* d_flag, const uint32_t* d_data, void* stream) {
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  if (v < 1 || v > 16) return fail(VSP_E_ARG, "v must be in [1, 16]");
  if (w < 1 || w > 1024) return fail(VSP_E_ARG, "w must be in [1, 1024]");
  if (((uint64_t)w << v) > kMaxLaunch) return fail(VSP_E_ARG, "w * 2^v must not exceed 2^22");
  VSP_HIP(hipSetDevice(ctx->device));
  vsp_status s;
  const uint64_t cells = (uint64_t)w << v;
  const size_t T0 = (LWE_N + 1) * 4, T1 = (RING_N + 1) * 4, TR = TRLWE_WORDS * 4;
  const size_t ram_b = cells * TR, addr_b = (size_t)v * TRGSW_WORDS * 4;
  if ((s = check_device_range(ctx, d_ram, ram_b, "d_ram"))) return s;
  if ((s = check_device_range(ctx, d_addr, addr_b, "d_addr"))) return s;
  if ((s = check_device_range(ctx, d_flag, T0, "d_flag"))) return s;
  if ((s = check_device_range(ctx, d_data, (size_t)w * T0, "d_data"))) return s;
  if ((s = check_no_overlap(d_ram, ram_b, d_addr, addr_b, "d_ram and d_addr"))) return s;
  if ((s = check_no_overlap(d_ram, ram_b, d_flag, T0, "d_ram and d_flag"))) return s;
  if ((s = check_no_overlap(d_ram, ram_b, d_data, (size_t)w * T0, "d_ram and d_data"))) return s;
  // scratch: selectors (C and G - C, NTT), torus G - C, read trees, control, bars, refresh
  if ((s = scratch_reserve(ctx, ctx->ntt_sel, (size_t)2 * v * TRGSW_NTT_U64 * 8))) return s;
  const size_t tree_b = (cells / 2 > 0 ? cells / 2 : 1) * TR;
  if ((s = scratch_reserve(ctx, ctx->mem_a, tree_b))) return s;
  if ((s = scratch_reserve(ctx, ctx->mem_b, tree_b))) return s;
  // mem_c: [gneg torus v TRGSW][src (1 + 2w) TLWE0][idx 3 * 2w u32][ops 2w][acc2 2w TRLWE][u w TRLWE]
  const size_t off_src = (size_t)v * TRGSW_WORDS * 4;
  const size_t off_idx = off_src + (1 + 2 * (size_t)w) * T0;
  const size_t off_ops = off_idx + 3 * 2 * (size_t)w * 4;
  const size_t off_acc = (off_ops + 2 * (size_t)w + 255) & ~(size_t)255;
  const size_t off_u = off_acc + 2 * (size_t)w * TR;
  const size_t mem_c_b = off_u + (size_t)w * TR;
  if ((s = scratch_reserve(ctx, ctx->mem_c, mem_c_b))) return s;
  // mem_d: tlwe0 [cells] then abar [cells]
  if ((s = scratch_reserve(ctx, ctx->mem_d, cells * T0 * 2))) return s;
  if ((s = scratch_reserve(ctx, ctx->tlwe1, cells * T1))) return s;
  // matrix-core workspace for the control and refresh bootstraps where the tuning picks those
  // forms (both write TRLWE outputs, so no accumulator area)
  const uint64_t nbr = std::max<uint64_t>(2 * (uint64_t)w, cells);
  const bool matrix =
      br_matrix_form(ctx->tune.br_waves(2 * (uint64_t)w)) || br_matrix_form(ctx->tune.br_waves(cells));
  if (matrix && (s = scratch_reserve(ctx, ctx->mf_work, mf_work_bytes(nbr, false)))) return s;
  void* mfw = matrix ? ctx->mf_work.ptr : nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* mc = static_cast<char*>(ctx->mem_c.ptr);
  uint64_t* sel = static_cast<uint64_t*>(ctx->ntt_sel.ptr);
  uint64_t* selneg = sel + (size_t)v * TRGSW_NTT_U64;
  uint32_t* gneg = reinterpret_cast<uint32_t*>(mc);
  uint32_t* src = reinterpret_cast<uint32_t*>(mc + off_src);
  uint32_t* idx = reinterpret_cast<uint32_t*>(mc + off_idx);
  uint8_t* ops = reinterpret_cast<uint8_t*>(mc + off_ops);
  uint32_t* acc2 = reinterpret_cast<uint32_t*>(mc + off_acc);
  uint32_t* u = reinterpret_cast<uint32_t*>(mc + off_u);
  uint32_t* t0 = static_cast<uint32_t*>(ctx->mem_d.ptr);
  uint32_t* abar = t0 + cells * (LWE_N + 1);
  uint32_t* t1 = static_cast<uint32_t*>(ctx->tlwe1.ptr);
  hipError_t e;
  // selectors
  if ((e = launch_gadget_minus(d_addr, gneg, v, st)) != hipSuccess) return hip_fail(e, "G - C");
  if ((e = launch_trgsw_to_ntt(ctx, d_addr, sel, v, st)) != hipSuccess) return hip_fail(e, "selector conversion");
  if ((e = launch_trgsw_to_ntt(ctx, gneg, selneg, v, st)) != hipSuccess) return hip_fail(e, "selector conversion");
  // read unit at the address: r_i -> src rows 1 + w + i
  uint32_t* res = nullptr;
  if ((e = run_trees(ctx, sel, v, 0, (int)v, d_ram, (1ull << v) * TRLWE_WORDS, 1, w, static_cast<uint32_t*>(ctx->mem_a.ptr),
                     static_cast<uint32_t*>(ctx->mem_b.ptr), &res, st)) != hipSuccess)
    return hip_fail(e, "read tree");
  if ((e = launch_sample_extract(res, t1, w, 1, st)) != hipSuccess) return hip_fail(e, "sample extract");
  if ((e = launch_keyswitch(ctx, nullptr, t1, nullptr, src + (1 + (size_t)w) * (LWE_N + 1), w, st)) != hipSuccess)
    return hip_fail(e, "key switch");
  // control unit: src = [f, x_0..x_{w-1}, r_0..r_{w-1}]; gates AND(f, x_i), ANDNOT(r_i, f)
  if ((e = hipMemcpyAsync(src, d_flag, T0, hipMemcpyDeviceToDevice, st)) != hipSuccess) return hip_fail(e, "copy flag");
  if ((e = hipMemcpyAsync(src + (LWE_N + 1), d_data, (size_t)w * T0, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return hip_fail(e, "copy data");
  if ((e = launch_ram_control_tables(idx, ops, w, st)) != hipSuccess) return hip_fail(e, "control tables");
  if ((e = launch_gate_prologue(ctx, ops, src, src, idx, idx + 2 * w, nullptr, abar, nullptr, 2 * (uint64_t)w, st,
                                false)) != hipSuccess)
    return hip_fail(e, "control prologue");
  if ((e = launch_blind_rotate(ctx, ops, abar, nullptr, acc2, 2 * (uint64_t)w, 0, st, nullptr, nullptr, nullptr,
                              mfw)) != hipSuccess)
    return hip_fail(e, "control bootstraps");
  if ((e = launch_ram_control(acc2, u, (int)w, st)) != hipSuccess) return hip_fail(e, "control combine");
  // write unit: bars, then refresh every cell with a bootstrap back to TRLWE, in place
  if ((e = launch_ram_bars(ctx, sel, selneg, d_ram, u, t1, (int)v, (int)w, st)) != hipSuccess) return hip_fail(e, "write bars");
  if ((e = launch_keyswitch(ctx, nullptr, t1, nullptr, t0, cells, st)) != hipSuccess) return hip_fail(e, "refresh key switch");
  if ((e = launch_gate_prologue_uniform(ctx, OP_IDENT, t0, abar, cells, st)) != hipSuccess) return hip_fail(e, "refresh prologue");
  if ((e = launch_blind_rotate(ctx, nullptr, abar, nullptr, d_ram, cells, 0, st, nullptr, nullptr, nullptr, mfw)) !=
      hipSuccess)
    return hip_fail(e, "refresh bootstraps");
  return VSP_OK;
}

}  // extern "C"
