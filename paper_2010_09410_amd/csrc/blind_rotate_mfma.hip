// Blind rotation on the matrix cores: every external product of a step is an exact integer
// matrix product over the whole batch, computed with int8 MFMA (Sec. 2.1.2, TRGSW and CMUX;
// the same accumulator recurrence as the NTT kernels, with the polynomial products done
// without a transform).
//
// For one TRGSW row r (gadget level k of ACC polynomial h, r = 3h + k) and output polynomial
// o, the product of the digit polynomial d with the key polynomial K in Z[X]/(X^N + 1) is
//   out[i] = sum_j d[j] Kt[i - j],   Kt[t] = K[t] (t >= 0), -K[t + N] (t < 0),
// a Toeplitz matrix-vector product. Over a batch of gates the digits form the rows of A
// (gates x (6 rows x N)), the key's Toeplitz blocks form B ((6 x N) x (2 x N)), and
// ACC += A B (mod 2^32) is one step. Exactness: the digits are in [-32, 31] and every key word
// is split into four balanced signed bytes Kt = sum_b 2^{8b} c_b (c_b in [-128, 127], mod
// 2^32); per byte plane the int32 sums are below 6 x 1024 x 32 x 128 < 2^25, and the planes
// are folded by Horner's rule in the accumulators (plane 3 first, shift by 8 bits between
// planes), the int32 wrap-around of the matrix cores being arithmetic mod 2^32.
//
// A step is two launches: k_mf_digits writes A for the step (bytes in the lane order of the
// MFMA operands), then k_mf_step computes the product for one tile of 32 gates and one output
// polynomial per workgroup and adds it to ACC. The B operand is never stored as a matrix: a
// 32 x 32 tile of a Toeplitz block depends only on its diagonal offset, so a lane reads its
// sixteen bytes straight from the extended key row Kt (staged in LDS), and moving to the next
// 32 input coefficients turns the tile of output block nb into that of block nb - 1, which
// the wave already holds: one new B operand per four matrix instructions.
#include "vsp_internal.h"

namespace vsp {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int MF_ROWS = 2 * GADGET_L;  // TRGSW rows
constexpr int MF_PLANES = 4;           // balanced bytes of a torus word
constexpr int MF_E = 2 * RING_N;       // extended row Kt[t - N], t in [0, 2N)
constexpr int MF_KB = RING_N / 32;     // 32-coefficient blocks of an input polynomial

// Digit-operand bytes of one tile of MF_TILE gates: [row r][block kb][lane][16].
constexpr size_t MF_A_TILE = (size_t)MF_TILE * MF_ROWS * RING_N;

// Key bytes per step: [row r][output o][plane b][t].
constexpr size_t MF_KEY_STEP = (size_t)MF_ROWS * 2 * MF_PLANES * MF_E;

// Extended key rows in balanced bytes: E[i][r][o][b][t] = byte b of Kt_{i,r,o}[t - N]
// (Kt[-N] = 0), from the torus key bk [n][2l][2][N].
__global__ __launch_bounds__(256) void k_mf_key(const u32* __restrict__ bk, int8_t* __restrict__ E, uint64_t rows) {
  const uint64_t id = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= rows * MF_E) return;
  const uint64_t row = id / MF_E;  // (i * 6 + r) * 2 + o
  const int t = (int)(id - row * MF_E);
  const int tau = t - RING_N;
  u32 v = 0;
  if (tau >= 0) v = bk[row * RING_N + tau];
  else if (tau > -RING_N) v = 0u - bk[row * RING_N + tau + RING_N];
  int8_t* out = E + row * MF_PLANES * MF_E + t;
#pragma unroll
  for (int b = 0; b < MF_PLANES; b++) {
    const int8_t c = (int8_t)(v & 255u);  // v = c (mod 256), c in [-128, 127]
    out[b * MF_E] = c;
    v = (v - (u32)(int32_t)c) >> 8;
  }
}

// ACC = (0, X^{-bbar} (mu, ..., mu)) for the gates that bootstrap.
__global__ __launch_bounds__(256) void k_mf_init(const uint8_t* __restrict__ ops, const u32* __restrict__ abar,
                                                  u32* __restrict__ acc, uint64_t B) {
  const uint64_t id = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= B * 2 * RING_N) return;
  const uint64_t g = id / (2 * RING_N);
  if (ops && !op_bootstraps(ops[g])) return;
  const int c = (int)(id - g * 2 * RING_N);
  const int bbar = (int)abar[g * TLWE0 + LWE_N];
  const int k0 = (2 * RING_N - bbar) & (2 * RING_N - 1);
  acc[id] = (c < RING_N) ? 0u : rotated_testvector(c - RING_N, k0);
}

// Digits of step i: for gate g, row r = 3h + k and coefficient j, digit k + 1 of
// (X^{abar_i} ACC_h - ACC_h)[j], written as the A operand of the step's products. Byte q of
// lane (m, kh) of block kb holds coefficient j = 32 kb + 16 kh + 15 - q of gate 32 mt + m
// (the order that makes the B bytes of a lane ascend in the key row). Gates at or above B and
// gates that do not bootstrap get zero digits.
// Workgroup (mt, h, eighth e of the gates): for each of its 8 gates, thread t takes
// coefficients 4t .. 4t + 3 (coalesced reads of ACC and of its rotation), and the bytes are
// gathered in LDS in operand order, then written out as 128-byte runs.
constexpr int MF_DG = 8;  // gates per digit workgroup

__global__ __launch_bounds__(256) void k_mf_digits(const uint8_t* __restrict__ ops, const u32* __restrict__ abar,
                                                    const u32* __restrict__ acc, int8_t* __restrict__ A, uint64_t B,
                                                    int step) {
  __shared__ u32 sA[GADGET_L][MF_KB][2 * MF_DG][4];
  const uint64_t mt = blockIdx.x;
  const int h = blockIdx.y, e = blockIdx.z, t = threadIdx.x;
  const int kb = t >> 3, kh = (t >> 2) & 1, dw = 3 - (t & 3);
  // all loads of the workgroup's gates first (their latencies overlap), then the digits
  bool live[MF_DG];
  int a[MF_DG];
  uint4 own[MF_DG];
  u32 rot[MF_DG][4];
#pragma unroll
  for (int mm = 0; mm < MF_DG; mm++) {
    const uint64_t g = mt * MF_TILE + (uint64_t)e * MF_DG + mm;
    live[mm] = g < B && (!ops || op_bootstraps(ops[g]));
    a[mm] = live[mm] ? (int)abar[g * TLWE0 + step] : 0;
  }
#pragma unroll
  for (int mm = 0; mm < MF_DG; mm++) {
    const uint64_t g = mt * MF_TILE + (uint64_t)e * MF_DG + mm;
    const u32* p = acc + (g * 2 + h) * RING_N;
    own[mm] = live[mm] ? reinterpret_cast<const uint4*>(p)[t] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int s = 0; s < 4; s++) {
      const int idx = (4 * t + 3 - s - a[mm]) & (2 * RING_N - 1);
      const u32 r = live[mm] ? p[idx & (RING_N - 1)] : 0u;
      rot[mm][s] = (idx & RING_N) ? 0u - r : r;
    }
  }
#pragma unroll
  for (int mm = 0; mm < MF_DG; mm++) {
    u32 w[GADGET_L] = {0u, 0u, 0u};
    if (live[mm]) {
      const u32 ov[4] = {own[mm].x, own[mm].y, own[mm].z, own[mm].w};
#pragma unroll
      for (int s = 0; s < 4; s++) {  // byte s of the lane's dword: coefficient 4t + 3 - s
        const u32 x = (rot[mm][s] - ov[3 - s]) + DECOMP_OFFSET;
#pragma unroll
        for (int k = 0; k < GADGET_L; k++)
          w[k] |= ((((x >> (32 - BG_BIT * (k + 1))) & 63u) - 32u) & 255u) << (8 * s);
      }
    }
#pragma unroll
    for (int k = 0; k < GADGET_L; k++) sA[k][kb][mm + MF_DG * kh][dw] = w[k];
  }
  __syncthreads();
  // out: rows 3h .. 3h + 2, blocks kb, lanes e*8 + (0..7) and 32 + e*8 + (0..7)
  const uint4* src = reinterpret_cast<const uint4*>(&sA[0][0][0][0]);
  uint4* dst = reinterpret_cast<uint4*>(A + mt * MF_A_TILE) + (size_t)GADGET_L * h * MF_KB * 64;
  for (int c = t; c < GADGET_L * MF_KB * 2 * MF_DG; c += 256) {
    const int ll = c % (2 * MF_DG), rk = c / (2 * MF_DG);  // rk = k * MF_KB + kb
    const int lane = (ll % MF_DG) + MF_DG * e + 32 * (ll / MF_DG);
    dst[(size_t)rk * 64 + lane] = src[c];
  }
}

// ACC[g][o] += (A B)[g][o] for the 32 gates of tile blockIdx.x and output polynomial
// o = blockIdx.y. Eight waves; wave w owns output coefficients [128 w, 128 w + 128) as four
// 32 x 32 blocks nb. Lane (n, kh) of the B operand of block nb at input block kb holds
// Kt[i - j] for i = 128 w + 32 nb + n and j = 32 kb + 16 kh + 15 - q, q = 0..15: the bytes
// E[t0 + q] with t0 = N + 128 w + 32 (nb - kb) + n - 16 kh - 15, in [1, 2032].
// The key row sits in LDS in sixteen copies, copy c shifted down by c bytes, so that the
// sixteen bytes from t0 are one aligned 16-byte read of copy t0 mod 16 (the same copy for a
// lane at every block kb, as t0 moves by 32).
// The 24 passes (plane b from 3 down, row r) each stage the tile's 32 KB of row-r digits and
// the copies of key row (r, o, b); the next pass's data is loaded into registers while the
// current pass computes, and stored to the other buffer after it. Within a pass, the LDS
// reads of block kb + 2 are issued before the four products of block kb; the B operands live
// in a ring of eight registers (block nb at kb in slot (nb - kb) mod 8), so the Toeplitz shift
// costs no moves.
constexpr int MF_A_PASS_U4 = MF_KB * 64;               // 16-byte operands per row and tile
constexpr int MF_PASSES = MF_PLANES * MF_ROWS;
constexpr int MF_COPY_U4 = MF_E / 16 + 1;               // one shifted copy and a 16-byte tail
constexpr int MF_ECOPIES_U4 = 16 * MF_COPY_U4;
constexpr size_t MF_STEP_LDS = 2 * (size_t)(MF_A_PASS_U4 + MF_ECOPIES_U4) * 16;

__global__ __launch_bounds__(512) void k_mf_step(const int8_t* __restrict__ Ek, const int8_t* __restrict__ A,
                                                  u32* __restrict__ acc, const uint8_t* __restrict__ ops,
                                                  uint64_t B) {
  extern __shared__ uint4 mf_lds[];
  uint4* abuf = mf_lds;                            // [2][MF_A_PASS_U4]
  uint4* ebuf = mf_lds + 2 * MF_A_PASS_U4;         // [2][16 copies][MF_COPY_U4]
  const uint64_t mt = blockIdx.x;
  const int o = blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, n = lane & 31, kh = lane >> 5;
  const int tb = RING_N + 128 * wave + n - 16 * kh - 15;
  const int cp = tb & 15;                          // this lane's key copy
  const int bofs = cp * MF_COPY_U4 + ((tb - cp) >> 4) - 2 * (MF_KB - 1);  // block kb, nb: + 2 (MF_KB - 1 - kb + nb)
  const uint4* Ag = reinterpret_cast<const uint4*>(A + mt * MF_A_TILE);
  const u32* Eu = reinterpret_cast<const u32*>(Ek);
  // pass p: plane b = 3 - p / 6, row r = p % 6; thread t stages dword t of every copy, which
  // needs dwords t .. t + 4 of the row (zero past its end)
  auto e_row = [&](int pass) {
    return Eu + (((size_t)(pass % MF_ROWS) * 2 + o) * MF_PLANES + (MF_PLANES - 1 - pass / MF_ROWS)) * (MF_E / 4);
  };
  auto stage_e = [&](uint4* dst, const u32 (&d)[5]) {
    u32* dw = reinterpret_cast<u32*>(dst);
#pragma unroll
    for (int c = 0; c < 16; c++)
      dw[c * MF_COPY_U4 * 4 + tid] = __builtin_amdgcn_alignbyte(d[(c >> 2) + 1], d[c >> 2], c & 3);
  };
  if (tid < 32) {  // the tails of the copies of both buffers
    ebuf[(tid >> 4) * MF_ECOPIES_U4 + (tid & 15) * MF_COPY_U4 + MF_E / 16] = make_uint4(0u, 0u, 0u, 0u);
  }
  {
    const uint4* as = Ag + tid;
    const uint4 x0 = as[0], x1 = as[512], x2 = as[1024], x3 = as[1536];
    const u32* er = e_row(0);
    u32 d[5];
#pragma unroll
    for (int q = 0; q < 5; q++) d[q] = (tid + q < MF_E / 4) ? er[tid + q] : 0u;
    abuf[tid] = x0;
    abuf[tid + 512] = x1;
    abuf[tid + 1024] = x2;
    abuf[tid + 1536] = x3;
    stage_e(ebuf, d);
  }
  __syncthreads();
  static_assert(MF_A_PASS_U4 == 4 * 512 && MF_E / 4 == 512, "four 16-byte loads and one key dword per thread and pass");
  v16i c[4];
#pragma unroll
  for (int nb = 0; nb < 4; nb++)
#pragma unroll
    for (int x = 0; x < 16; x++) c[nb][x] = 0;
  auto run_pass = [&](int pass) {
    const int buf = pass & 1;
    const int nx = (pass + 1 < MF_PASSES) ? pass + 1 : pass;  // the last pass fetches itself again, unused
    const uint4* as = Ag + (size_t)(nx % MF_ROWS) * MF_A_PASS_U4 + tid;
    const uint4 p0 = as[0], p1 = as[512], p2 = as[1024], p3 = as[1536];
    u32 pd[5];
    {
      const u32* er = e_row(nx);
#pragma unroll
      for (int q = 0; q < 5; q++) pd[q] = (tid + q < MF_E / 4) ? er[tid + q] : 0u;
    }
    const uint4* Ar = abuf + buf * MF_A_PASS_U4 + lane;
    const uint4* Bp = ebuf + buf * MF_ECOPIES_U4 + bofs;
    v4i R[8], Av[4];
    auto ld = [](const uint4& u) { return v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w}; };
#pragma unroll
    for (int nb = 0; nb < 4; nb++) R[nb] = ld(Bp[2 * (MF_KB - 1 + nb)]);
    R[7] = ld(Bp[2 * (MF_KB - 2)]);  // B_0 of block 1
    Av[0] = ld(Ar[0]);
    Av[1] = ld(Ar[64]);
    for (int k8 = 0; k8 < MF_KB; k8 += 8) {
#pragma unroll
      for (int s8 = 0; s8 < 8; s8++) {
        // reads for block kb + 2 (the last two blocks re-read the last one, unused)
        const int kb = k8 + s8;
        const int kn = (kb + 2 < MF_KB) ? kb + 2 : MF_KB - 1;
        Av[(s8 + 2) & 3] = ld(Ar[kn * 64]);
        R[(6 - s8) & 7] = ld(Bp[2 * (MF_KB - 1 - kn)]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int nb = 0; nb < 4; nb++)
          c[nb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Av[s8 & 3], R[(nb - s8) & 7], c[nb], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (pass % MF_ROWS == MF_ROWS - 1 && pass + 1 < MF_PASSES) {
#pragma unroll
      for (int nb = 0; nb < 4; nb++)
#pragma unroll
        for (int x = 0; x < 16; x++) c[nb][x] = (int)((u32)c[nb][x] << 8);
    }
    // the other buffer was last read in the previous pass, before the barrier that ended it
    if (pass + 1 < MF_PASSES) {
      uint4* ad = abuf + (buf ^ 1) * MF_A_PASS_U4 + tid;
      ad[0] = p0;
      ad[512] = p1;
      ad[1024] = p2;
      ad[1536] = p3;
      stage_e(ebuf + (buf ^ 1) * MF_ECOPIES_U4, pd);
    }
    __syncthreads();
  };
  for (int pass = 0; pass < MF_PASSES - 1; pass++) run_pass(pass);
  // result (m, i): lane n + 32 kh, register x: m = 8 (x / 4) + 4 kh + x % 4, i = 128 w + 32 nb + n.
  // The accumulator words are loaded before the last pass and updated after it.
  u32 av[16][4];
  bool live[16];
#pragma unroll
  for (int x = 0; x < 16; x++) {
    const uint64_t g = mt * MF_TILE + 8 * (x >> 2) + 4 * kh + (x & 3);
    live[x] = g < B && (!ops || op_bootstraps(ops[g]));
    const u32* p = acc + (g * 2 + o) * RING_N + 128 * wave + n;
#pragma unroll
    for (int nb = 0; nb < 4; nb++) av[x][nb] = live[x] ? p[32 * nb] : 0u;
  }
  run_pass(MF_PASSES - 1);
#pragma unroll
  for (int x = 0; x < 16; x++) {
    if (!live[x]) continue;
    const uint64_t g = mt * MF_TILE + 8 * (x >> 2) + 4 * kh + (x & 3);
    u32* p = acc + (g * 2 + o) * RING_N + 128 * wave + n;
#pragma unroll
    for (int nb = 0; nb < 4; nb++) p[32 * nb] = av[x][nb] + (u32)c[nb][x];
  }
}

hipError_t init_mf_kernel_attributes() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_step), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)MF_STEP_LDS);
}

size_t mf_key_bytes() { return (size_t)LWE_N * MF_KEY_STEP; }

size_t mf_work_bytes(uint64_t B, bool need_acc) {
  const uint64_t tiles = (B + MF_TILE - 1) / MF_TILE;
  return tiles * MF_A_TILE + (need_acc ? (size_t)B * 2 * RING_N * 4 : 0);
}

hipError_t launch_mf_key(const uint32_t* bk, int8_t* E, hipStream_t st) {
  const uint64_t rows = (uint64_t)LWE_N * MF_ROWS * 2;
  hipLaunchKernelGGL(k_mf_key, dim3((unsigned)((rows * MF_E + 255) / 256)), dim3(256), 0, st, bk, E, rows);
  return hipGetLastError();
}

hipError_t launch_blind_rotate_mfma(const vsp_context* ctx, const uint8_t* ops, const uint32_t* abar, uint32_t* tlwe1,
                                    uint32_t* trlwe, uint64_t B, void* work, hipStream_t st) {
  if (B == 0) return hipSuccess;
  const uint64_t tiles = (B + MF_TILE - 1) / MF_TILE;
  int8_t* A = static_cast<int8_t*>(work);
  u32* acc = trlwe ? trlwe : reinterpret_cast<u32*>(A + tiles * MF_A_TILE);
  hipLaunchKernelGGL(k_mf_init, dim3((unsigned)((B * 2 * RING_N + 255) / 256)), dim3(256), 0, st, ops, abar, acc, B);
  for (int i = 0; i < LWE_N; i++) {
    hipLaunchKernelGGL(k_mf_digits, dim3((unsigned)tiles, 2, MF_TILE / MF_DG), dim3(256), 0, st, ops, abar, acc, A, B,
                       i);
    hipLaunchKernelGGL(k_mf_step, dim3((unsigned)tiles, 2), dim3(512), MF_STEP_LDS, st,
                       ctx->mf_key + (size_t)i * MF_KEY_STEP, A, acc, ops, B);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && tlwe1) e = launch_sample_extract(acc, tlwe1, B, 1, st);
  return e;
}

}  // namespace vsp
