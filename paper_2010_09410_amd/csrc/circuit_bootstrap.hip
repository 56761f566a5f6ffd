// Circuit bootstrapping on the GPU (Sec. 2.1.2 "Circuit Bootstrapping"; the CMUX memory needs
// it for its address bits, Sec. 8.2, and the paper's GPU library lacked it because its moduli
// exceed 64 bits, Sec. 6.2(a)). A level-0 TLWE of a bit becomes a level-1 TRGSW (l x 2^6
// gadget): for each gadget level j = 1..l, a level-2 blind rotation over the 2^64 torus
// (degree N2 = 2048, gadget l2 = 4 x 2^9) with the test vector 1/(2 Bg^j), SampleExtract at 0
// plus 1/(2 Bg^j), then two private functional key switches to level-1 TRLWE (x -> -s1 x and
// x -> x) that give TRGSW rows j-1 and l+j-1.
//
// Exact level-2 products. A product d(X) K(X) in Z[X]/(X^2048 + 1) with gadget digits |d| <=
// 2^8 and 64-bit torus key words is computed as two products with the key's 32-bit halves
// (K = K_lo + 2^32 K_hi): each has integer coefficients below 8 rows x 2048 x 2^8 x 2^32 =
// 2^54 < p/2, so the wave-level NTT modulo p = 2^64 - 2^32 + 1 of the level-1 path yields them
// exactly; the low half is lifted to a signed 64-bit integer, the high half mod 2^32, and the
// torus result is lo + 2^32 hi mod 2^64. Degree 2048 reuses the degree-1024 transform through
// the even/odd split a(X) = a_e(X^2) + X a_o(X^2): with Y = X^2 (Y^1024 = -1),
//   (d K)_e = d_e K_e + Y d_o K_o,   (d K)_o = d_e K_o + d_o K_e,
// products in Z[Y]/(Y^1024 + 1). The key is stored transformed, with Y folded into Y K_o.
#include "vsp_internal.h"

namespace vsp {

constexpr int CB_N2 = 2048;
constexpr int CB_L2 = 4;
constexpr int CB_BG2 = 9;
constexpr int CB_ROWS = 2 * CB_L2;       // level-2 TRGSW rows
constexpr int CB_T = 12;                 // private key-switch digits
constexpr int CB_BB = 2;                 // private key-switch base bits
constexpr int CB_TLWE2 = CB_N2 + 1;
// Transformed key per (step, row, output o, half-word w): [slot s][lane][2] u64.
constexpr size_t CB_KEY_BLOCK = (size_t)32 * 64 * 2;
constexpr size_t CB_KEY_STEP = (size_t)CB_ROWS * 2 * 2 * CB_KEY_BLOCK;
// Private key-switching keys: [u][k <= N2][p < t][v - 1 < 3][2][N] u32.
constexpr size_t CB_PKS_ROW = (size_t)2 * RING_N;
constexpr size_t CB_PKS_U = (size_t)CB_TLWE2 * CB_T * 3 * CB_PKS_ROW;
// Rounding offset of the level-2 gadget decomposition: sum_r (Bg2/2) 2^(64 - 9r) + 2^(64 - 36 - 1).
constexpr u64 cb_decomp_offset() {
  u64 o = 0;
  for (int r = 1; r <= CB_L2; r++) o += (u64)(1u << (CB_BG2 - 1)) << (64 - CB_BG2 * r);
  return o + (1ull << (64 - CB_BG2 * CB_L2 - 1));
}
constexpr u64 CB_DECOMP_OFFSET = cb_decomp_offset();

// Exact signed lift of a canonical residue, as a 64-bit two's-complement word.
__device__ __forceinline__ u64 gl_lift_u64(u64 c) { return c > (GL_P >> 1) ? c - GL_P : c; }

// Inverse transform with the 64-bit lift: out[t] = coefficient l + 32 t of N times the
// polynomial, the exact integer in (-p/2, p/2) as a two's-complement word (the twist sign
// of coefficients t >= 1 as in ntt_inverse_lift).
__device__ __forceinline__ void ntt_inverse_lift64(u64 (&v)[32], const u64* ti, u32* reg, int l, u64 (&out)[32]) {
  dft32_inverse(v);
  table_multiply(v, ti, l);
  transpose_inverse(v, reg, l);
  dft32_inverse(v);
  out[0] = gl_lift_u64(gl_canon(v[0]));
#pragma unroll
  for (int t = 1; t < 32; t++) out[t] = 0ull - gl_lift_u64(gl_mul_pow2(v[t], 96 - 3 * t));
}

// Key conversion: one wave per (step i, row, output o, half-word w). Half h of the wave
// transforms the h-part (even / odd coefficients) of the key word; lane l of half 0 stores
// (K_e, Y K_o) and of half 1 (K_o, K_e) for each slot, scaled by 1/1024.
__global__ __launch_bounds__(256) void k_cb_key(const u64* __restrict__ bk2, u64* __restrict__ dst,
                                                const u64* __restrict__ tw, u64 ninv, uint64_t jobs) {
  __shared__ u32 lds[4 * WAVE_T_U32];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t job = (uint64_t)blockIdx.x * 4 + wave;
  if (job >= jobs) return;
  const int lane = threadIdx.x & 63, l = lane & 31, h = lane >> 5;
  const int w = (int)(job & 1);
  const uint64_t poly = job >> 1;  // (i * 8 + row) * 2 + o
  const u64* K = bk2 + poly * CB_N2;
  u32* reg = lds + wave * WAVE_T_U32 + h * TREGION;
  u64 v[32], y[32];
#pragma unroll
  for (int t = 0; t < 32; t++) {
    const u64 word = K[2 * (l + 32 * t) + h];
    v[t] = w ? (word >> 32) : (word & 0xFFFFFFFFull);
    y[t] = (l == 1 && t == 0) ? 1ull : 0ull;
  }
  ntt_forward(v, tw, reg, l);
  ntt_forward(y, tw, reg, l);
  u64* out = dst + job * CB_KEY_BLOCK;
#pragma unroll
  for (int s = 0; s < 32; s++) {
    u64 ke, ko;
    both_halves(v[s], ke, ko);
    const u64 e0 = h ? ko : ke;
    const u64 e1 = h ? ke : gl_mul(y[s], ko);
    out[((size_t)s * 64 + lane) * 2] = gl_canon(gl_mul(e0, ninv));
    out[((size_t)s * 64 + lane) * 2 + 1] = gl_canon(gl_mul(e1, ninv));
  }
}

// Level-2 blind rotation, one workgroup of four waves per job (circuit bootstrap c = job / l,
// gadget level j = job % l + 1), the accumulator in global memory (L2-resident). Per step, for
// each ACC polynomial h: wave r forms gadget digit r + 1 of X^abar ACC_h - ACC_h (lanes 0-31 the
// even coefficients, 32-63 the odd ones) and transforms it into its LDS block; then wave
// q = 2 o + w accumulates, for output o and key half-word w, sum_r (D_e, D_o) x (entries of its
// lane). After both polynomials, each wave inverts its sums; the high-word waves pass theirs
// through their own LDS blocks and the low-word waves add lo + 2^32 hi to ACC_o. A wave's
// transpose region lies in its own LDS block (used before the block is filled, and after it
// has been read), so a workgroup takes 80 KiB of LDS and two fit on a compute unit. The
// result is SampleExtract_0 + 1/(2 Bg^j) as a TLWE2.
constexpr int CB_THREADS = 256;
constexpr size_t CB_BLOCK_U64 = (size_t)32 * 64;              // one wave's transformed digits: 16 KiB
constexpr size_t CB_LDS = (4 * CB_BLOCK_U64 + 2048) * 8;       // digit blocks + twiddle tables: 80 KiB
static_assert((size_t)WAVE_T_U32 <= 2 * CB_BLOCK_U64 && (size_t)2 * CB_N2 / 2 <= 2 * CB_BLOCK_U64,
              "transpose region and high-word exchange fit in one block");
constexpr int CB_KCH = 4;  // key slots per chunk of the streamed key

__global__ __launch_bounds__(CB_THREADS, 2) void k_cb_rotate(const u64* __restrict__ key, const u64* __restrict__ tw,
                                                           const u32* __restrict__ in, u64* __restrict__ accbuf,
                                                           u64* __restrict__ out, int gadget_l, int bgbit) {
  extern __shared__ u64 cb_lds[];
  u64* dig = cb_lds;                                           // [4][32][64]
  u64* tws = dig + 4 * CB_BLOCK_U64;                           // forward then inverse tables
  const uint64_t job = blockIdx.x;
  const int j = (int)(job % (uint64_t)gadget_l) + 1;
  const u32* c = in + (job / (uint64_t)gadget_l) * TLWE0;
  u64* acc = accbuf + job * 2 * CB_N2;                         // [2][N2]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l = lane & 31, half = lane >> 5;
  u64* myblock = dig + (size_t)wave * CB_BLOCK_U64;
  u32* reg = reinterpret_cast<u32*>(myblock) + half * TREGION;
  const u64 tvv = 1ull << (63 - bgbit * j);                    // 1/(2 Bg^j)
  for (int i = tid; i < 2048; i += CB_THREADS) tws[i] = tw[i];
  {
    const u32 bbar = ((c[LWE_N] + (1u << 19)) >> 20) & (2 * CB_N2 - 1);
    const int k = (int)((2 * CB_N2 - bbar) & (2 * CB_N2 - 1));
    for (int m = tid; m < CB_N2; m += CB_THREADS) {
      const bool neg = (m < (k & (CB_N2 - 1))) != (k >= CB_N2);
      acc[m] = 0;
      acc[CB_N2 + m] = neg ? (0ull - tvv) : tvv;
    }
  }
  __syncthreads();
  const int o = wave >> 1, wd = wave & 1;
  for (int i = 0; i < LWE_N; i++) {
    const int abar = (int)(((c[i] + (1u << 19)) >> 20) & (2 * CB_N2 - 1));
    const u64* kstep = key + (size_t)i * CB_KEY_STEP;
    u64 sum[32];
#pragma unroll
    for (int s = 0; s < 32; s++) sum[s] = 0;
#pragma unroll 1
    for (int h = 0; h < 2; h++) {
      const u64* P = acc + h * CB_N2;
      {
        u64 x[32];
        const int sh = 64 - CB_BG2 * (wave + 1);
        // the accumulator words come from L2 in four groups of eight coefficients (bounded
        // registers in flight)
#pragma unroll
        for (int t8 = 0; t8 < 32; t8 += 8) {
#pragma unroll
          for (int t = t8; t < t8 + 8; t++) {
            const int m = 2 * (l + 32 * t) + half;
            const int src = (m - abar) & (2 * CB_N2 - 1);
            const u64 r = P[src & (CB_N2 - 1)];
            const u64 d = ((src & CB_N2) ? (0ull - r) : r) - P[m];
            x[t] = (u64)((int64_t)(((d + CB_DECOMP_OFFSET) >> sh) & ((1u << CB_BG2) - 1)) - (1 << (CB_BG2 - 1)));
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        ntt_forward<true>(x, tws, reg, l);
#pragma unroll
        for (int s = 0; s < 32; s++) myblock[(size_t)s * 64 + lane] = x[s];
      }
      __syncthreads();
      // key entries stream in chunks of CB_KCH slots, the next chunk (of this row or the
      // next) in flight while the current one is used
      auto key_row = [&](int r) {
        return reinterpret_cast<const ulonglong2*>(kstep + ((((size_t)(h * CB_L2 + r)) * 2 + o) * 2 + wd) *
                                                               CB_KEY_BLOCK) + lane;
      };
      ulonglong2 kc[CB_KCH];
      {
        const ulonglong2* kb = key_row(0);
#pragma unroll
        for (int q = 0; q < CB_KCH; q++) kc[q] = kb[q * 64];
      }
#pragma unroll 1
      for (int r = 0; r < CB_L2; r++) {
        const ulonglong2* kb = key_row(r);
        const ulonglong2* kb_next = key_row(r + 1 < CB_L2 ? r + 1 : r);
        const u64* dr = dig + (size_t)r * CB_BLOCK_U64;
#pragma unroll
        for (int cc = 0; cc < 32 / CB_KCH; cc++) {
          ulonglong2 kn[CB_KCH];
#pragma unroll
          for (int q = 0; q < CB_KCH; q++)
            kn[q] = (cc + 1 < 32 / CB_KCH) ? kb[(CB_KCH * (cc + 1) + q) * 64] : kb_next[q * 64];
#pragma unroll
          for (int q = 0; q < CB_KCH; q++) {
            const int sl = CB_KCH * cc + q;
            sum[sl] = gl_add(sum[sl], gl_dot2(dr[sl * 64 + l], kc[q].x, dr[sl * 64 + 32 + l], kc[q].y));
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int q = 0; q < CB_KCH; q++) kc[q] = kn[q];
        }
      }
      __syncthreads();
    }
    u64 z[32];
    ntt_inverse_lift64(sum, tws + 1024, reg, l, z);
    // the high word of output o goes through the LDS block of wave 2 o + 1 (its own)
    u32* xch = reinterpret_cast<u32*>(dig + (size_t)(2 * o + 1) * CB_BLOCK_U64);
    if (wd == 1) {
#pragma unroll
      for (int t = 0; t < 32; t++) xch[2 * (l + 32 * t) + half] = (u32)z[t];
    }
    __syncthreads();
    if (wd == 0) {
      u64* A = acc + o * CB_N2;
#pragma unroll
      for (int t = 0; t < 32; t++) {
        const int m = 2 * (l + 32 * t) + half;
        A[m] += z[t] + ((u64)xch[m] << 32);
      }
    }
    __syncthreads();
  }
  u64* dst = out + job * CB_TLWE2;
  for (int m = tid; m < CB_N2; m += CB_THREADS) dst[m] = (m == 0) ? acc[0] : (0ull - acc[CB_N2 - m]);
  if (tid == 0) dst[CB_N2] = acc[CB_N2] + tvv;
}

// Latency form of the level-2 blind rotation: one workgroup of eight waves per job, so that a
// step's eight digit rows are transformed at once (wave w: polynomial h = w / 4, digit
// w % 4 + 1, into its own LDS block) and the key products are split by polynomial (wave w:
// output o and half-word wd of c = w % 4 = 2 o + wd over the rows of h = w / 4). The sums of
// h = 1 then go through the LDS blocks of waves 4-7 to waves 0-3, which invert them and update
// ACC as in k_cb_rotate. 144 KiB of LDS, one workgroup per compute unit: for batches that the
// four-wave form would run in a single round anyway, where each step's critical path is then
// one transform and four rows of key products instead of two and eight.
constexpr int CBW_THREADS = 512;
constexpr size_t CBW_LDS = (8 * CB_BLOCK_U64 + 2048) * 8;  // digit blocks + twiddle tables: 144 KiB

__global__ __launch_bounds__(CBW_THREADS, 1) void k_cb_rotate_wide(const u64* __restrict__ key,
                                                                  const u64* __restrict__ tw,
                                                                  const u32* __restrict__ in,
                                                                  u64* __restrict__ accbuf, u64* __restrict__ out,
                                                                  int gadget_l, int bgbit) {
  extern __shared__ u64 cb_lds[];
  u64* dig = cb_lds;                                           // [8][32][64]
  u64* tws = dig + 8 * CB_BLOCK_U64;                           // forward then inverse tables
  const uint64_t job = blockIdx.x;
  const int j = (int)(job % (uint64_t)gadget_l) + 1;
  const u32* c = in + (job / (uint64_t)gadget_l) * TLWE0;
  u64* acc = accbuf + job * 2 * CB_N2;                         // [2][N2]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l = lane & 31, half = lane >> 5;
  u64* myblock = dig + (size_t)wave * CB_BLOCK_U64;
  u32* reg = reinterpret_cast<u32*>(myblock) + half * TREGION;
  const u64 tvv = 1ull << (63 - bgbit * j);                    // 1/(2 Bg^j)
  for (int i = tid; i < 2048; i += CBW_THREADS) tws[i] = tw[i];
  {
    const u32 bbar = ((c[LWE_N] + (1u << 19)) >> 20) & (2 * CB_N2 - 1);
    const int k = (int)((2 * CB_N2 - bbar) & (2 * CB_N2 - 1));
    for (int m = tid; m < CB_N2; m += CBW_THREADS) {
      const bool neg = (m < (k & (CB_N2 - 1))) != (k >= CB_N2);
      acc[m] = 0;
      acc[CB_N2 + m] = neg ? (0ull - tvv) : tvv;
    }
  }
  __syncthreads();
  const int h = wave >> 2, cw = wave & 3, o = cw >> 1, wd = cw & 1;
  for (int i = 0; i < LWE_N; i++) {
    const int abar = (int)(((c[i] + (1u << 19)) >> 20) & (2 * CB_N2 - 1));
    const u64* kstep = key + (size_t)i * CB_KEY_STEP;
    {
      const u64* P = acc + h * CB_N2;
      u64 x[32];
      const int sh = 64 - CB_BG2 * (cw + 1);
#pragma unroll
      for (int t8 = 0; t8 < 32; t8 += 8) {
#pragma unroll
        for (int t = t8; t < t8 + 8; t++) {
          const int m = 2 * (l + 32 * t) + half;
          const int src = (m - abar) & (2 * CB_N2 - 1);
          const u64 r = P[src & (CB_N2 - 1)];
          const u64 d = ((src & CB_N2) ? (0ull - r) : r) - P[m];
          x[t] = (u64)((int64_t)(((d + CB_DECOMP_OFFSET) >> sh) & ((1u << CB_BG2) - 1)) - (1 << (CB_BG2 - 1)));
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      ntt_forward<true>(x, tws, reg, l);
#pragma unroll
      for (int s = 0; s < 32; s++) myblock[(size_t)s * 64 + lane] = x[s];
    }
    __syncthreads();
    u64 sum[32];
#pragma unroll
    for (int s = 0; s < 32; s++) sum[s] = 0;
    {
      auto key_row = [&](int r) {
        return reinterpret_cast<const ulonglong2*>(kstep + ((((size_t)(h * CB_L2 + r)) * 2 + o) * 2 + wd) *
                                                               CB_KEY_BLOCK) + lane;
      };
      ulonglong2 kc[CB_KCH];
      {
        const ulonglong2* kb = key_row(0);
#pragma unroll
        for (int q = 0; q < CB_KCH; q++) kc[q] = kb[q * 64];
      }
#pragma unroll 1
      for (int r = 0; r < CB_L2; r++) {
        const ulonglong2* kb = key_row(r);
        const ulonglong2* kb_next = key_row(r + 1 < CB_L2 ? r + 1 : r);
        const u64* dr = dig + (size_t)(h * CB_L2 + r) * CB_BLOCK_U64;
#pragma unroll
        for (int cc = 0; cc < 32 / CB_KCH; cc++) {
          ulonglong2 kn[CB_KCH];
#pragma unroll
          for (int q = 0; q < CB_KCH; q++)
            kn[q] = (cc + 1 < 32 / CB_KCH) ? kb[(CB_KCH * (cc + 1) + q) * 64] : kb_next[q * 64];
#pragma unroll
          for (int q = 0; q < CB_KCH; q++) {
            const int sl = CB_KCH * cc + q;
            sum[sl] = gl_add(sum[sl], gl_dot2(dr[sl * 64 + l], kc[q].x, dr[sl * 64 + 32 + l], kc[q].y));
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int q = 0; q < CB_KCH; q++) kc[q] = kn[q];
        }
      }
    }
    __syncthreads();  // every digit block is read
    if (h == 1) {
#pragma unroll
      for (int s = 0; s < 32; s++) myblock[(size_t)s * 64 + lane] = sum[s];
    }
    __syncthreads();
    u64 z[32];
    u32* xch = reinterpret_cast<u32*>(dig + (size_t)(2 * o + 1) * CB_BLOCK_U64);
    if (h == 0) {
      const u64* other = dig + (size_t)(4 + cw) * CB_BLOCK_U64;
#pragma unroll
      for (int s = 0; s < 32; s++) sum[s] = gl_add(sum[s], other[(size_t)s * 64 + lane]);
      ntt_inverse_lift64(sum, tws + 1024, reg, l, z);
      // the high word of output o goes through the LDS block of wave 2 o + 1 (its own)
      if (wd == 1) {
#pragma unroll
        for (int t = 0; t < 32; t++) xch[2 * (l + 32 * t) + half] = (u32)z[t];
      }
    }
    __syncthreads();
    if (h == 0 && wd == 0) {
      u64* A = acc + o * CB_N2;
#pragma unroll
      for (int t = 0; t < 32; t++) {
        const int m = 2 * (l + 32 * t) + half;
        A[m] += z[t] + ((u64)xch[m] << 32);
      }
    }
    __syncthreads();
  }
  u64* dst = out + job * CB_TLWE2;
  for (int m = tid; m < CB_N2; m += CBW_THREADS) dst[m] = (m == 0) ? acc[0] : (0ull - acc[CB_N2 - m]);
  if (tid == 0) dst[CB_N2] = acc[CB_N2] + tvv;
}

// Private functional key switch: out = sum_{k <= N2, p < t2} PKSK[u][k][p][v_{k,p} - 1] over the
// nonzero base-4 digits v_{k,p} (most significant first) of c_k rounded to 24 bits. Row u = 0
// is TRGSW row j - 1, u = 1 row l + j - 1. Row-stationary: workgroup (tile of G jobs, u, slice
// of 256 output words), thread t owning word 256 slice + t; for every (k, p) it loads the three
// key words of its column once and adds the one each job's digit selects, so the key is read
// once per tile instead of once per job (sums mod 2^32 in any order: the same bits). The
// rounded coefficients of the tile's jobs are staged in LDS a chunk of k at a time.
constexpr int CBP_CHUNK = 32;
template <int G>
__global__ __launch_bounds__(256, 2) void k_cb_privks(const u32* __restrict__ pksk, const u64* __restrict__ tl2,
                                                   u32* __restrict__ out, int gadget_l, uint64_t jobs) {
  __shared__ u32 chat[CBP_CHUNK][G];
  __shared__ u32 tab[CB_T][4][256];  // thread t's column: entry v of digit p (v = 0: zero)
  const uint64_t j0 = (uint64_t)blockIdx.x * G;
  const int u = blockIdx.y, tid = threadIdx.x, col = (int)blockIdx.z * 256 + tid;
  const int ng = (int)((jobs - j0 < (uint64_t)G) ? jobs - j0 : (uint64_t)G);
  constexpr int TB = CB_T * CB_BB;
  const u32* key = pksk + (size_t)u * CB_PKS_U + col;
  u32 a[G];
#pragma unroll
  for (int g = 0; g < G; g++) a[g] = 0u;
#pragma unroll
  for (int p = 0; p < CB_T; p++) tab[p][0][tid] = 0u;
  for (int k0 = 0; k0 < CB_TLWE2; k0 += CBP_CHUNK) {
    __syncthreads();  // the previous chunk is consumed
    for (int i = tid; i < CBP_CHUNK * G; i += 256) {
      const int kk = i / G, g = i % G;
      u32 v = 0u;
      if (g < ng && k0 + kk < CB_TLWE2)
        v = (u32)((tl2[(j0 + g) * CB_TLWE2 + k0 + kk] + (1ull << (64 - TB - 1))) >> (64 - TB));
      chat[kk][g] = v;
    }
    __syncthreads();
    const int kn = (CB_TLWE2 - k0 < CBP_CHUNK) ? CB_TLWE2 - k0 : CBP_CHUNK;
    for (int kk = 0; kk < kn; kk++) {
      const u32* kr = key + (size_t)(k0 + kk) * CB_T * 3 * CB_PKS_ROW;
      u32 c[G];  // the jobs' rounded coefficients: the same in every lane
#pragma unroll
      for (int g = 0; g < G; g++) c[g] = __builtin_amdgcn_readfirstlane(chat[kk][g]);
      // the thread's own column goes to LDS, where a wave-uniform digit indexes it (no compare
      // and select per job and digit; each thread reads only what it wrote, so no barrier)
#pragma unroll
      for (int p = 0; p < CB_T; p++)
#pragma unroll
        for (int v = 0; v < 3; v++) tab[p][v + 1][tid] = kr[(size_t)(p * 3 + v) * CB_PKS_ROW];
#pragma unroll
      for (int p = 0; p < CB_T; p++)
#pragma unroll
        for (int g = 0; g < G; g++) a[g] += tab[p][(c[g] >> (CB_BB * (CB_T - 1 - p))) & 3u][tid];
    }
  }
  for (int g = 0; g < ng; g++) {
    const uint64_t job = j0 + g;
    const int j = (int)(job % (uint64_t)gadget_l) + 1;
    const int row = u == 0 ? j - 1 : gadget_l + j - 1;
    out[((job / (uint64_t)gadget_l) * 2 * gadget_l + row) * CB_PKS_ROW + col] = a[g];
  }
}

hipError_t init_cb_kernel_attributes() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cb_rotate),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)CB_LDS);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cb_rotate_wide), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)CBW_LDS);
  return e;
}

}  // namespace vsp

using namespace vsp;

struct vsp_cbkey {
  vsp_context* ctx = nullptr;
  u64* key = nullptr;   // transformed level-2 bootstrapping key
  u32* pksk = nullptr;  // private key-switching keys
  Scratch tl2;          // TLWE2 outputs of the blind rotations
  Scratch acc;          // their accumulators [job][2][N2]
  int form = 0;         // level-2 blind rotation: 0 by batch size, 1 four-wave form, 2 eight-wave form
};

extern "C" {

vsp_status vsp_cbkey_create(vsp_context* ctx, const uint64_t* bk2_host, const uint32_t* pksk_host, vsp_cbkey** out) {
  if (out == nullptr) return fail(VSP_E_ARG, "out is NULL");
  *out = nullptr;
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  if (bk2_host == nullptr || pksk_host == nullptr) return fail(VSP_E_ARG, "bk2_host and pksk_host must not be NULL");
  VSP_HIP(hipSetDevice(ctx->device));
  VSP_HIP(init_cb_kernel_attributes());
  auto* k = new vsp_cbkey();
  k->ctx = ctx;
  u64* tmp = nullptr;
  auto bail = [&](vsp_status st) {
    if (tmp) (void)hipFree(tmp);
    vsp_cbkey_destroy(k);
    return st;
  };
  const size_t bk2_bytes = (size_t)LWE_N * CB_ROWS * 2 * CB_N2 * 8;
  const size_t pksk_bytes = 2 * CB_PKS_U * 4;
  hipError_t e;
  if ((e = hipMalloc(&tmp, bk2_bytes)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(level-2 key)"));
  if ((e = hipMalloc(&k->key, (size_t)LWE_N * CB_KEY_STEP * 8)) != hipSuccess)
    return bail(hip_fail(e, "hipMalloc(level-2 key, transformed)"));
  if ((e = hipMalloc(&k->pksk, pksk_bytes)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(private key-switching keys)"));
  if ((e = hipMemcpy(tmp, bk2_host, bk2_bytes, hipMemcpyHostToDevice)) != hipSuccess) return bail(hip_fail(e, "upload"));
  if ((e = hipMemcpy(k->pksk, pksk_host, pksk_bytes, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(hip_fail(e, "upload"));
  const uint64_t jobs = (uint64_t)LWE_N * CB_ROWS * 2 * 2;
  const u64 ninv = gl_powmod_const(RING_N, GL_P - 2);
  hipLaunchKernelGGL(k_cb_key, dim3((unsigned)((jobs + 3) / 4)), dim3(256), 0, nullptr, tmp, k->key, ctx->tw, ninv,
                     jobs);
  if ((e = hipGetLastError()) != hipSuccess) return bail(hip_fail(e, "level-2 key conversion"));
  if ((e = hipDeviceSynchronize()) != hipSuccess) return bail(hip_fail(e, "level-2 key conversion"));
  (void)hipFree(tmp);
  tmp = nullptr;
  *out = k;
  return VSP_OK;
}

vsp_status vsp_cbkey_destroy(vsp_cbkey* k) {
  if (k == nullptr) return VSP_OK;
  (void)hipSetDevice(k->ctx->device);
  (void)hipDeviceSynchronize();
  for (void* p : {(void*)k->key, (void*)k->pksk, k->tl2.ptr, k->acc.ptr})
    if (p) (void)hipFree(p);
  delete k;
  return VSP_OK;
}

vsp_status vsp_cbkey_set_form(vsp_cbkey* key, int form) {
  if (key == nullptr) return fail(VSP_E_ARG, "key is NULL");
  if (form < 0 || form > 2) return fail(VSP_E_ARG, "form must be 0 (by batch size), 1 (four waves) or 2 (eight waves)");
  key->form = form;
  return VSP_OK;
}

vsp_status vsp_circuit_bootstrap(vsp_context* ctx, vsp_cbkey* key, const uint32_t* d_in, uint32_t* d_out, uint64_t R,
                                 void* stream) {
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  vsp_status s = VSP_OK;
  if (key == nullptr || key->ctx != ctx) return fail(VSP_E_ARG, "key is NULL or belongs to another context");
  if (R == 0) return VSP_OK;
  if (R > (1ull << 20)) return fail(VSP_E_ARG, "R too large");
  VSP_HIP(hipSetDevice(ctx->device));
  const size_t ib = (size_t)R * TLWE0 * 4, ob = (size_t)R * 2 * GADGET_L * 2 * RING_N * 4;
  if ((s = check_device_range(ctx, d_in, ib, "d_in"))) return s;
  if ((s = check_device_range(ctx, d_out, ob, "d_out"))) return s;
  if ((s = check_no_overlap(d_out, ob, d_in, ib, "d_out and d_in"))) return s;
  const uint64_t jobs = R * GADGET_L;
  if ((s = scratch_reserve(ctx, key->tl2, jobs * CB_TLWE2 * 8))) return s;
  if ((s = scratch_reserve(ctx, key->acc, jobs * 2 * CB_N2 * 8))) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  u64* tl2 = static_cast<u64*>(key->tl2.ptr);
  // the eight-wave form while the jobs fit one workgroup per compute unit (the four-wave form,
  // two per compute unit, would run them in one round too, each step on half the waves)
  const bool wide = key->form == 2 || (key->form == 0 && jobs <= (uint64_t)(ctx->cus > 0 ? ctx->cus : 256));
  if (wide)
    hipLaunchKernelGGL(k_cb_rotate_wide, dim3((unsigned)jobs), dim3(CBW_THREADS), CBW_LDS, st, key->key, ctx->tw, d_in,
                       static_cast<u64*>(key->acc.ptr), tl2, GADGET_L, BG_BIT);
  else
    hipLaunchKernelGGL(k_cb_rotate, dim3((unsigned)jobs), dim3(CB_THREADS), CB_LDS, st, key->key, ctx->tw, d_in,
                       static_cast<u64*>(key->acc.ptr), tl2, GADGET_L, BG_BIT);
  // tiles as large as keep about four workgroups per compute unit busy (16 per tile and u)
  const uint64_t slices = CB_PKS_ROW / 256;
  auto tiles = [&](uint64_t g) { return (jobs + g - 1) / g; };
  const uint64_t want = 4ull * (uint64_t)(ctx->cus > 0 ? ctx->cus : 256);
  if (tiles(32) * 2 * slices >= want)
    hipLaunchKernelGGL(k_cb_privks<32>, dim3((unsigned)tiles(32), 2, (unsigned)slices), dim3(256), 0, st, key->pksk,
                       tl2, d_out, GADGET_L, jobs);
  else if (tiles(16) * 2 * slices >= want)
    hipLaunchKernelGGL(k_cb_privks<16>, dim3((unsigned)tiles(16), 2, (unsigned)slices), dim3(256), 0, st, key->pksk,
                       tl2, d_out, GADGET_L, jobs);
  else if (tiles(8) * 2 * slices >= want)
    hipLaunchKernelGGL(k_cb_privks<8>, dim3((unsigned)tiles(8), 2, (unsigned)slices), dim3(256), 0, st, key->pksk,
                       tl2, d_out, GADGET_L, jobs);
  else
    hipLaunchKernelGGL(k_cb_privks<2>, dim3((unsigned)tiles(2), 2, (unsigned)slices), dim3(256), 0, st, key->pksk,
                       tl2, d_out, GADGET_L, jobs);
  VSP_HIP(hipGetLastError());
  return VSP_OK;
}

}  // extern "C"
