// Blind rotation on the matrix cores: every external product of a step is an exact integer
// matrix product over the whole batch, computed with int8 MFMA (Sec. 2.1.2, TRGSW and CMUX;
// the same accumulator recurrence as the NTT kernels, with the polynomial products done
// without a transform).
//
// For one TRGSW row r (gadget level k of ACC polynomial h, r = 3h + k) and output polynomial
// o, the product of the digit polynomial x with the key polynomial K in Z[X]/(X^N + 1) is
//   y[i] = sum_j x[j] Kt[i - j],   Kt[t] = K[t] (t >= 0), -K[t + N] (t < 0),
// a Toeplitz matrix-vector product y = T x. With T split into blocks of N/2 (T11 = T00 for a
// Toeplitz matrix) and x = (x0, x1), one level of the Karatsuba split needs three products of
// size N/2 instead of four:
//   P1 = T00 (x0 + x1),  P2 = (T01 - T00) x1,  P3 = (T10 - T00) x0,
//   y0 = P1 + P2,        y1 = P1 + P3,
// each again Toeplitz, with the sequences S1[t] = Kt[t], S2[t] = Kt[t - N/2] - Kt[t],
// S3[t] = Kt[t + N/2] - Kt[t] for t in (-N/2, N/2). Over a batch the operands (x0 + x1, x1,
// x0) of all gates form the rows of A, and the three Toeplitz blocks per (row, output) form
// a block-diagonal B: 3/4 of the multiply-adds of the plain product.
// Exactness: the operands carry the digits plus 32, x' = x + 32 in [0, 63] (x0' + x1' in
// [0, 126]), which keeps the top bits of every operand byte clear and so lowers the switching
// activity, and with it the power, of the matrix pipes; key words are split into four balanced
// signed bytes Kt = sum_b 2^{8b} c_b (c_b in [-128, 127], mod 2^32); per byte plane the int32
// sums stay below 6 x 512 x 126 x 128 < 2^26, and the planes are folded by Horner's rule in
// the accumulators (plane 3 first, shift by 8 bits between planes), the int32 wrap-around of
// the matrix cores being arithmetic mod 2^32. The offset adds 32 times the product of the row
// key with the all-ones polynomial to each row's product, a vector that depends on the key
// only: with K' the sum of the six row keys of output o, (K' (1 + X + .. + X^{N-1}))[i] =
// 2 S_i - S_{N-1} in Z[X]/(X^N + 1) for the prefix sums S_i = K'[0] + .. + K'[i], so
// C[i] = 64 S_i - 32 S_{N-1} is stored per (step, output) with the key and taken off where a
// step's shares are combined.
//
// A step is one launch of k_mf_step: for one tile of 32 gates and one output polynomial per
// workgroup it computes P1, P2 and P3, combines them, adds y to ACC, and writes the next
// step's A rows that depend on that polynomial (bytes in the lane order of the MFMA
// operands; segments 1 and 2 only, segment 0 being their bytewise sum, formed when a step
// stages its operands). k_mf_digits writes the first step's A (all three segments, which the
// split form reads). B is never stored
// as a matrix: a 32 x 32 tile of a Toeplitz block depends only on its diagonal offset, so a
// lane reads its sixteen bytes straight from the sequence (staged in LDS), and moving to the
// next 32 input coefficients turns the tile of output block nb into that of block nb - 1,
// which the wave already holds: one new B operand per four matrix instructions.
#include "vsp_internal.h"

namespace vsp {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int MF_ROWS = 2 * GADGET_L;   // TRGSW rows
constexpr int MF_PLANES = 4;            // balanced bytes of a torus word
constexpr int MF_HALF = RING_N / 2;     // size of the three sub-products
constexpr int MF_SUB = 3;               // sub-products P1, P2, P3
constexpr int MF_S = RING_N;            // sequence S_s[t - N/2], t in [0, N) (t = 0 unused)
constexpr int MF_KB = MF_HALF / 32;     // 32-coefficient blocks of a sub-product's input

// Digit-operand bytes of one tile of MF_TILE gates: [row r][segment s][block kb][lane][16],
// segment 0 holding x0 + x1, 1 x1, 2 x0 (the inputs of P1, P2, P3).
constexpr size_t MF_A_ROW = (size_t)MF_SUB * MF_KB * 64 * 16;
constexpr size_t MF_A_TILE = (size_t)MF_ROWS * MF_A_ROW;

// Key bytes per step: [row r][output o][plane b][sub-product s][t]; after the n steps, the
// offset corrections C[step][o][N] (uint32).
constexpr size_t MF_KEY_STEP = (size_t)MF_ROWS * 2 * MF_PLANES * MF_SUB * MF_S;
constexpr size_t MF_KEY_BYTES = (size_t)LWE_N * MF_KEY_STEP;
constexpr int MF_CORR_STEP_U32 = 2 * RING_N;
constexpr int MF_OFS = 1 << (BG_BIT - 1);  // added to every digit in the operands: (x >> sh) & 63 is digit + 32

// The correction words of output o of the step whose key bytes start key_off bytes into the
// key at base.
__device__ __forceinline__ const u32* mf_corr(const int8_t* base, uint64_t key_off, int o) {
  return reinterpret_cast<const u32*>(base + MF_KEY_BYTES) + (key_off / MF_KEY_STEP) * MF_CORR_STEP_U32 +
         (size_t)o * RING_N;
}

// The three sequences of every (step, row, output) in balanced bytes, from the torus key
// bk [n][2l][2][N]: E[i][r][o][b][s][t] = byte b of S_s[t - N/2].
__device__ __forceinline__ u32 kt_word(const u32* K, int t) {  // Kt[t], t in (-N, N)
  return t >= 0 ? K[t] : 0u - K[t + RING_N];
}

__global__ __launch_bounds__(256) void k_mf_key(const u32* __restrict__ bk, int8_t* __restrict__ E, uint64_t rows) {
  const uint64_t id = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= rows * MF_S) return;
  const uint64_t row = id / MF_S;  // (i * 6 + r) * 2 + o
  const int t = (int)(id - row * MF_S);
  const int tau = t - MF_HALF;
  const u32* K = bk + row * RING_N;
  u32 v[MF_SUB] = {0u, 0u, 0u};
  if (t > 0) {
    const u32 k0 = kt_word(K, tau);
    v[0] = k0;
    v[1] = kt_word(K, tau - MF_HALF) - k0;
    v[2] = kt_word(K, tau + MF_HALF) - k0;
  }
  int8_t* out = E + row * MF_PLANES * MF_SUB * MF_S + t;
#pragma unroll
  for (int s = 0; s < MF_SUB; s++) {
    u32 w = v[s];
#pragma unroll
    for (int b = 0; b < MF_PLANES; b++) {
      const int8_t c = (int8_t)(w & 255u);  // w = c (mod 256), c in [-128, 127]
      out[((size_t)b * MF_SUB + s) * MF_S] = c;
      w = (w - (u32)(int32_t)c) >> 8;
    }
  }
}

// Offset corrections: workgroup (step, o) sums the six row keys of output o (K'), scans the
// sum, and writes C[i] = 64 S_i - 32 S_{N-1} (S_i = K'[0] + .. + K'[i], all mod 2^32).
// Thread t takes coefficients 4t .. 4t + 3.
static_assert(RING_N == 4 * 256, "four coefficients per thread");
__global__ __launch_bounds__(256) void k_mf_corr(const u32* __restrict__ bk, u32* __restrict__ C) {
  __shared__ u32 part[256];
  const int step = blockIdx.x, o = blockIdx.y, t = threadIdx.x;
  u32 v[4] = {0u, 0u, 0u, 0u};
  for (int r = 0; r < MF_ROWS; r++) {
    const uint4 k = reinterpret_cast<const uint4*>(bk + (((size_t)step * MF_ROWS + r) * 2 + o) * RING_N)[t];
    v[0] += k.x;
    v[1] += k.y;
    v[2] += k.z;
    v[3] += k.w;
  }
  v[1] += v[0];
  v[2] += v[1];
  v[3] += v[2];
  part[t] = v[3];
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {  // inclusive scan of the per-thread sums
    const u32 add = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  const u32 before = t > 0 ? part[t - 1] : 0u, total = part[255];
  uint4 c;
  constexpr u32 two = 2u * MF_OFS, one = MF_OFS;
  c.x = two * (before + v[0]) - one * total;
  c.y = two * (before + v[1]) - one * total;
  c.z = two * (before + v[2]) - one * total;
  c.w = two * (before + v[3]) - one * total;
  reinterpret_cast<uint4*>(C + ((size_t)step * 2 + o) * RING_N)[t] = c;
}

// ACC = (0, X^{-bbar} (mu, ..., mu)) for the gates that bootstrap; with `zero` non-NULL also
// clears the same rows there (the first step's target in the rotating-buffer split form).
__global__ __launch_bounds__(256) void k_mf_init(const uint8_t* __restrict__ ops, const u32* __restrict__ abar,
                                                  u32* __restrict__ acc, uint64_t B, u32* __restrict__ zero) {
  const uint64_t id = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= B * 2 * RING_N) return;
  if (zero) zero[id] = 0u;
  const uint64_t g = id / (2 * RING_N);
  if (ops && !op_bootstraps(ops[g])) return;
  const int c = (int)(id - g * 2 * RING_N);
  const int bbar = (int)abar[g * TLWE0 + LWE_N];
  const int k0 = (2 * RING_N - bbar) & (2 * RING_N - 1);
  acc[id] = (c < RING_N) ? 0u : rotated_testvector(c - RING_N, k0);
}

// Digits of step i: for gate g, row r = 3h + k and coefficient j, digit k + 1 of
// x = (X^{abar_i} ACC_h - ACC_h) plus MF_OFS, written as the A operand of the step's products:
// segment 1 holds x1 = x[N/2 ..], segment 2 x0 = x[.. N/2], segment 0 their sum. In a segment,
// byte q of lane (m, kh) of block kb holds local coefficient j = 32 kb + 16 kh + 15 - q of gate
// 32 mt + m (the order that makes the B bytes of a lane ascend in the key sequence). Gates
// at or above B and gates that do not bootstrap get zero bytes (their products are dropped).
// Workgroup (mt, h, eighth e of the gates): thread t takes local coefficients 4 jg .. 4 jg + 3
// (jg = t mod 128) of both halves for gates t / 128, t / 128 + 2, ... (coalesced reads of ACC
// and of its rotation); the bytes are gathered in LDS in operand order, then written out as
// 128-byte runs.
// The digit bytes of one (gate, quad of local coefficients jg, level k) for the three segments
// (packed four coefficients per word as in the operand layout), from the rotated and plain
// values of both halves.
__device__ __forceinline__ void mf_digit_words(const u32 (&rot0)[4], const u32 (&own0)[4], const u32 (&rot1)[4],
                                               const u32 (&own1)[4], u32 (&w)[GADGET_L][MF_SUB]) {
#pragma unroll
  for (int s = 0; s < 4; s++) {  // byte s of the word: local coefficient 4 jg + 3 - s
    const u32 x0 = (rot0[s] - own0[3 - s]) + DECOMP_OFFSET;
    const u32 x1 = (rot1[s] - own1[3 - s]) + DECOMP_OFFSET;
#pragma unroll
    for (int k = 0; k < GADGET_L; k++) {
      const int sh = 32 - BG_BIT * (k + 1);
      const u32 d0 = (x0 >> sh) & 63u, d1 = (x1 >> sh) & 63u;  // digits plus MF_OFS
      w[k][0] |= ((d0 + d1) & 255u) << (8 * s);
      w[k][1] |= (d1 & 255u) << (8 * s);
      w[k][2] |= (d0 & 255u) << (8 * s);
    }
  }
}

constexpr int MF_DG = 8;  // gates per digit workgroup
// Shares of one (tile, output, sub-product, workgroup group) in the partial-sum split form:
// [gate m][local output i], N/2 words per gate.
constexpr size_t MF_PART_U32 = (size_t)MF_TILE * MF_HALF;

// With PG > 0 the step's shares are first added into ACC (the partial-sum split form, PG
// workgroups per (tile, output, sub-product)): y0[i] = sum over groups of P1[i] + P2[i],
// y1[i] = sum of P1[i] + P3[i] from the share blocks of output polynomial h, and ACC_h += y
// is written back. The updated polynomials of the workgroup's gates are staged in LDS, where
// the rotated coefficients are read. step == n: the shares of the last step only. DG gates
// per workgroup (8 for the first step of the fused form; the split form takes 4, or 2 with
// partial sums, for more workgroups on its latency-bound launches).
template <int PG, int DG = MF_DG>
__global__ __launch_bounds__(256) void k_mf_digits(const uint8_t* __restrict__ ops, const u32* __restrict__ abar,
                                                    u32* __restrict__ acc, int8_t* __restrict__ A, uint64_t B,
                                                    int step, const u32* __restrict__ part) {
  // the gates' polynomials h [DG][N] while digits are formed, then the operand words
  // sA[k][segment][kb][lane][4] gathered in operand order
  constexpr int SP_U4 = DG * RING_N / 4, SA_U4 = GADGET_L * MF_SUB * MF_KB * 2 * DG;
  __shared__ uint4 lds[SP_U4 > SA_U4 ? SP_U4 : SA_U4];
  const uint64_t mt = blockIdx.x;
  const int h = blockIdx.y, e = blockIdx.z, t = threadIdx.x;
  const int jg = t & 127, kb = jg >> 3, kh = (jg >> 2) & 1, dw = 3 - (jg & 3);
  constexpr int ROUNDS = DG / 2;
  bool live[ROUNDS];
  uint4 own[ROUNDS][2];
#pragma unroll
  for (int q = 0; q < ROUNDS; q++) {
    const int mm = 2 * q + (t >> 7);
    const uint64_t g = mt * MF_TILE + (uint64_t)e * DG + mm;
    live[q] = g < B && (!ops || op_bootstraps(ops[g]));
    uint4* p = reinterpret_cast<uint4*>(acc + (g * 2 + h) * RING_N);
#pragma unroll
    for (int half = 0; half < 2; half++)
      own[q][half] = live[q] ? p[half * (MF_HALF / 4) + jg] : make_uint4(0u, 0u, 0u, 0u);
    if (PG > 0 && live[q]) {
      const uint4* Q = reinterpret_cast<const uint4*>(part) +
                       ((mt * 2 + h) * MF_SUB * PG * MF_TILE + (uint64_t)e * DG + mm) * (MF_HALF / 4) + jg;
      constexpr size_t SUB_U4 = (size_t)PG * MF_PART_U32 / 4, RG_U4 = MF_PART_U32 / 4;
#pragma unroll
      for (int rg = 0; rg < (PG > 0 ? PG : 1); rg++) {
        const uint4 p1 = Q[rg * RG_U4], p2 = Q[SUB_U4 + rg * RG_U4], p3 = Q[2 * SUB_U4 + rg * RG_U4];
        own[q][0].x += p1.x + p2.x; own[q][0].y += p1.y + p2.y; own[q][0].z += p1.z + p2.z; own[q][0].w += p1.w + p2.w;
        own[q][1].x += p1.x + p3.x; own[q][1].y += p1.y + p3.y; own[q][1].z += p1.z + p3.z; own[q][1].w += p1.w + p3.w;
      }
      p[jg] = own[q][0];
      p[MF_HALF / 4 + jg] = own[q][1];
    }
    lds[mm * (RING_N / 4) + jg] = own[q][0];
    lds[mm * (RING_N / 4) + MF_HALF / 4 + jg] = own[q][1];
  }
  if (step >= LWE_N) return;  // uniform: the last step's shares only
  __syncthreads();
  u32 w[ROUNDS][GADGET_L][MF_SUB];
#pragma unroll
  for (int q = 0; q < ROUNDS; q++) {
    const int mm = 2 * q + (t >> 7);
    const uint64_t g = mt * MF_TILE + (uint64_t)e * DG + mm;
#pragma unroll
    for (int k = 0; k < GADGET_L; k++)
#pragma unroll
      for (int sg = 0; sg < MF_SUB; sg++) w[q][k][sg] = 0u;
    if (live[q]) {
      const int a = (int)abar[g * TLWE0 + step];
      const u32* P = reinterpret_cast<const u32*>(lds + mm * (RING_N / 4));
      u32 rot[2][4];
#pragma unroll
      for (int half = 0; half < 2; half++)
#pragma unroll
        for (int s = 0; s < 4; s++) {
          const int idx = (half * MF_HALF + 4 * jg + 3 - s - a) & (2 * RING_N - 1);
          const u32 r = P[idx & (RING_N - 1)];
          rot[half][s] = (idx & RING_N) ? 0u - r : r;
        }
      const u32 ov0[4] = {own[q][0].x, own[q][0].y, own[q][0].z, own[q][0].w};
      const u32 ov1[4] = {own[q][1].x, own[q][1].y, own[q][1].z, own[q][1].w};
      mf_digit_words(rot[0], ov0, rot[1], ov1, w[q]);
    }
  }
  __syncthreads();  // the staged polynomials are read: the region now gathers operand words
  u32(*sA)[MF_SUB][MF_KB][2 * DG][4] = reinterpret_cast<u32(*)[MF_SUB][MF_KB][2 * DG][4]>(lds);
#pragma unroll
  for (int q = 0; q < ROUNDS; q++) {
    const int mm = 2 * q + (t >> 7);
#pragma unroll
    for (int k = 0; k < GADGET_L; k++)
#pragma unroll
      for (int sg = 0; sg < MF_SUB; sg++) sA[k][sg][kb][mm + DG * kh][dw] = w[q][k][sg];
  }
  __syncthreads();
  // out: rows 3h .. 3h + 2, every segment and block, lanes e*8 + (0..7) and 32 + e*8 + (0..7)
  const uint4* src = lds;
  uint4* dst = reinterpret_cast<uint4*>(A + mt * MF_A_TILE + (size_t)GADGET_L * h * MF_A_ROW);
  for (int c = t; c < SA_U4; c += 256) {
    const int ll = c % (2 * DG), rk = c / (2 * DG);  // rk = (k * 3 + segment) * MF_KB + kb
    const int lane = (ll % DG) + DG * e + 32 * (ll / DG);
    dst[(size_t)rk * 64 + lane] = src[c];
  }
}

// The 64 products of one pass for a wave's four output blocks nb over the 16 input blocks kb
// of its segment. Block (nb, kb) takes the A operand of block kb (lane bytes at Ar[64 kb]) and
// the B operand of diagonal d = nb - kb (ldb(8 (MF_KB - 1 + d)): the Toeplitz tile depends on
// d only). The products are issued along diagonals: group t = 0..15 takes kb = t + nb for the
// four nb, four independent accumulators that share one B operand (d = -t) while A changes,
// A being the operand with the fewer switching bits (digits plus offset, against random key
// bytes); the products with kb >= 16 wrap to kb - 16 (d = 16 - t: 3, 2, 1 in the last three
// groups; the order of the integer sums does not matter). Each group loads the A operand of
// block t + 4 (first used by the next group) and the B operand of group t + 2; the wrapped
// products' operands are loaded two groups ahead.
template <typename LDB, typename LDA>
__device__ __forceinline__ void mf_pass_products(v16i (&c)[4], const uint4* __restrict__ Ar, LDB&& ldb, LDA&& lda) {
  v4i Av[8], Bm[3], Aw[3], Bx[3];
#pragma unroll
  for (int k = 0; k < 4; k++) Av[k] = lda(Ar[k * 64]);
  Bm[0] = ldb(8 * (MF_KB - 1));
  Bm[1] = ldb(8 * (MF_KB - 2));
#pragma unroll
  for (int t = 0; t < MF_KB; t++) {
    if (t + 4 < MF_KB) Av[(t + 4) & 7] = lda(Ar[(t + 4) * 64]);
    if (t + 2 < MF_KB) Bm[(t + 2) % 3] = ldb(8 * (MF_KB - 3 - t));
    if (t >= MF_KB - 5 && t < MF_KB - 2) {
      const int w = t - (MF_KB - 5);  // wrapped block w, diagonal 3 - w
      Aw[w] = lda(Ar[w * 64]);
      Bx[w] = ldb(8 * (MF_KB + 2 - w));
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      const int kb = t + nb;
      if (kb < MF_KB)
        c[nb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Av[kb & 7], Bm[t % 3], c[nb], 0, 0, 0);
      else
        c[nb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Aw[kb >= MF_KB ? kb - MF_KB : 0],
                                                      Bx[t >= MF_KB - 3 ? t - (MF_KB - 3) : 0], c[nb], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ACC[g][o] += y for the 32 gates of tile blockIdx.x and output polynomial o = blockIdx.y.
// Twelve waves: wave w computes sub-product s = w / 4 for local outputs
// [128 (w mod 4), 128 (w mod 4) + 128) as four 32 x 32 blocks nb. Lane (n, kh) of the B
// operand of block nb at input block kb holds S_s[i - j] for i = 128 (w mod 4) + 32 nb + n and
// j = 32 kb + 16 kh + 15 - q, q = 0..15: the bytes E_s[t0 + q] with
// t0 = N/2 + 128 (w mod 4) + 32 (nb - kb) + n - 16 kh - 15, in [1, 1008].
// Each sequence sits in LDS in four copies, copy c shifted down by c bytes, so that the
// sixteen bytes from t0 are four aligned words of copy t0 mod 4 (the same copy for a lane at
// every block kb, as t0 moves by 32).
// The 24 passes (plane b from 3 down, the six rows r) each stage the tile's 48 KB of row-r operands and
// the copies of the three sequences (r, o, b); the next pass's data is loaded into registers
// while the current pass computes, and stored to the other buffer after it. Within a pass the
// products run in the diagonal order of mf_pass_products. At the end P1 goes through LDS to
// the waves of P2 and P3, which form y0 = P1 + P2 and y1 = P1 + P3, take off the offset
// correction and write y to LDS; the workgroup adds y to ACC and keeps the updated polynomial
// in LDS, where the next step's digits are formed.
constexpr int MF_WAVES = 12;
constexpr int MF_THREADS = MF_WAVES * 64;
constexpr int MF_A_PASS_U4 = (int)(MF_A_ROW / 16);      // 3072 16-byte operands per row and tile
constexpr int MF_PASSES = MF_PLANES * MF_ROWS;
// one shifted copy (256 words read) padded to 264 words: 264 = 8 (mod 32), so the 32 lanes of
// a word read (copies t0 mod 4, words t0 / 4 over eight consecutive values) hit 32 banks
constexpr int MF_COPY_U32 = MF_S / 4 + 8;
constexpr int MF_ECOPIES_U32 = MF_SUB * 4 * MF_COPY_U32;
constexpr size_t MF_PASS_LDS = 2 * ((size_t)MF_A_PASS_U4 * 16 + (size_t)MF_ECOPIES_U32 * 4);
constexpr int MF_PROW = RING_N + 1;
constexpr size_t MF_POLY_LDS = (size_t)MF_TILE * MF_PROW * 4;
constexpr size_t MF_STEP_LDS = MF_PASS_LDS > MF_POLY_LDS ? MF_PASS_LDS : MF_POLY_LDS;
static_assert(MF_A_PASS_U4 == 4 * MF_THREADS && MF_SUB * MF_S / 4 == MF_THREADS,
              "four 16-byte operands and one key word per thread and pass");
static_assert((size_t)4 * 4 * 16 * 64 * 4 <= 2 * (size_t)MF_A_PASS_U4 * 16, "P1 fits in the operand buffers");

// Row of pass p: the six rows of a byte plane in any order give the same plane sum, so odd
// planes take them backwards and the rows a plane ends with are still in L2 when the next
// one starts.
__device__ __forceinline__ int mf_pass_row(int pass) {
  const int r = pass % MF_ROWS;
  return ((pass / MF_ROWS) & 1) ? MF_ROWS - 1 - r : r;
}

// Step kernel (Ek0, or the tile's tkeys entry, is the start of a whole key; key_off selects the
// step). With next_step >= 0 the workgroup then writes the digit operands of step
// next_step for rows 3o .. 3o + 2 of its tile into Anext: they depend only on the updated
// polynomial o of its own 32 gates, which it has just written, so no other workgroup is
// involved (the other output polynomial's workgroup writes rows 3(1 - o) ..).
__global__ __launch_bounds__(MF_THREADS) void k_mf_step(const int8_t* __restrict__ Ek0, const int8_t* __restrict__ A,
                                                         u32* __restrict__ acc, const uint8_t* __restrict__ ops,
                                                         uint64_t B, int8_t* __restrict__ Anext,
                                                         const u32* __restrict__ abar, int next_step,
                                                         const int8_t* const* __restrict__ tkeys, uint64_t key_off) {
  extern __shared__ uint4 mf_lds[];
  // the step's key: the context's (Ek0), or the tile's key set's
  const int8_t* __restrict__ Kb = tkeys ? tkeys[blockIdx.x] : Ek0;
  const int8_t* __restrict__ Ek = Kb + key_off;
  uint4* abuf = mf_lds;                                            // [2][MF_A_PASS_U4]
  u32* ebuf = reinterpret_cast<u32*>(mf_lds + 2 * MF_A_PASS_U4);  // [2][3 sequences][4 copies][MF_COPY_U32]
  const uint64_t mt = blockIdx.x;
  const int o = blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, n = lane & 31, kh = lane >> 5;
  const int sub = wave >> 2, wl = wave & 3;
  const int tb = MF_HALF + 128 * wl + n - 16 * kh - 15;
  const int cp = tb & 3;                                           // this lane's key copy
  // word offset of block kb, nb: + 8 (MF_KB - 1 - kb + nb)
  const int bofs = (sub * 4 + cp) * MF_COPY_U32 + ((tb - cp) >> 2) - 8 * (MF_KB - 1);
  const uint4* Ag = reinterpret_cast<const uint4*>(A + mt * MF_A_TILE);
  const u32* Eu = reinterpret_cast<const u32*>(Ek);
  // pass p: plane b = 3 - p / 6, row r = p % 6. Thread t stages word t mod 256 of the copies of
  // sequence t / 256, which needs words t mod 256 and the next one (zero past the end).
  const int es = tid >> 8, ew = tid & 255;
  auto e_row = [&](int pass) {
    return Eu + ((((size_t)mf_pass_row(pass) * 2 + o) * MF_PLANES + (MF_PLANES - 1 - pass / MF_ROWS)) * MF_SUB + es) *
                    (MF_S / 4);
  };
  auto stage_e = [&](u32* dst, u32 d0, u32 d1) {
#pragma unroll
    for (int c = 0; c < 4; c++) dst[(es * 4 + c) * MF_COPY_U32 + ew] = __builtin_amdgcn_alignbyte(d1, d0, c);
  };
  if (tid < 2 * MF_SUB * 4 * 4) {  // the tails of all copies of both buffers
    const int bufi = tid / (MF_SUB * 16), rest = tid % (MF_SUB * 16);
    ebuf[bufi * MF_ECOPIES_U32 + (rest >> 2) * MF_COPY_U32 + MF_S / 4 + (rest & 3)] = 0u;
  }
  // Only segments 1 and 2 (x1, x0 plus offset) are read from A: segment 0, their sum, is formed
  // while staging, a 32-bit add of packed bytes that cannot carry (each byte sum is at most
  // 126), so a row moves 32 KiB instead of 48 and the tile's rows stay in L2 across planes.
  // Thread t stages operand i = t of each segment, and threads t < 256 also i = t + 768.
  constexpr int SEG_U4 = MF_KB * 64;
  const bool two = tid < SEG_U4 - MF_THREADS;  // wave-uniform
  auto load_row = [&](const uint4* row, uint4 (&v)[4]) {
    v[0] = row[SEG_U4 + tid];
    v[1] = row[2 * SEG_U4 + tid];
    v[2] = v[3] = make_uint4(0u, 0u, 0u, 0u);
    if (two) {
      v[2] = row[SEG_U4 + MF_THREADS + tid];
      v[3] = row[2 * SEG_U4 + MF_THREADS + tid];
    }
  };
  auto store_row = [&](uint4* dst, const uint4 (&v)[4]) {
    auto sum = [](const uint4& a, const uint4& b) { return make_uint4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); };
    dst[tid] = sum(v[0], v[1]);
    dst[SEG_U4 + tid] = v[0];
    dst[2 * SEG_U4 + tid] = v[1];
    if (two) {
      dst[MF_THREADS + tid] = sum(v[2], v[3]);
      dst[SEG_U4 + MF_THREADS + tid] = v[2];
      dst[2 * SEG_U4 + MF_THREADS + tid] = v[3];
    }
  };
  static_assert(MF_A_PASS_U4 == MF_SUB * SEG_U4 && SEG_U4 - MF_THREADS <= MF_THREADS, "two rounds cover a segment");
  {
    uint4 x[4];
    load_row(Ag, x);
    const u32* er = e_row(0);
    const u32 d0 = er[ew], d1 = (ew + 1 < MF_S / 4) ? er[ew + 1] : 0u;
    store_row(abuf, x);
    stage_e(ebuf, d0, d1);
  }
  __syncthreads();
  v16i c[4];
#pragma unroll
  for (int nb = 0; nb < 4; nb++)
#pragma unroll
    for (int x = 0; x < 16; x++) c[nb][x] = 0;
  for (int pass = 0; pass < MF_PASSES; pass++) {
    const int buf = pass & 1;
    const int nx = (pass + 1 < MF_PASSES) ? pass + 1 : pass;  // the last pass fetches itself again, unused
    uint4 pa[4];
    load_row(Ag + (size_t)mf_pass_row(nx) * MF_A_PASS_U4, pa);
    u32 pd0, pd1;
    {
      const u32* er = e_row(nx);
      pd0 = er[ew];
      pd1 = (ew + 1 < MF_S / 4) ? er[ew + 1] : 0u;
    }
    const uint4* Ar = abuf + buf * MF_A_PASS_U4 + sub * (MF_KB * 64) + lane;
    const u32* Bp = ebuf + buf * MF_ECOPIES_U32 + bofs;
    auto ldb = [&](int wofs) {
      return v4i{(int)Bp[wofs], (int)Bp[wofs + 1], (int)Bp[wofs + 2], (int)Bp[wofs + 3]};
    };
    auto lda = [](const uint4& u) { return v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w}; };
    mf_pass_products(c, Ar, ldb, lda);
    if (pass % MF_ROWS == MF_ROWS - 1 && pass + 1 < MF_PASSES) {
#pragma unroll
      for (int nb = 0; nb < 4; nb++)
#pragma unroll
        for (int x = 0; x < 16; x++) c[nb][x] = (int)((u32)c[nb][x] << 8);
    }
    // the other buffer was last read in the previous pass, before the barrier that ended it
    if (pass + 1 < MF_PASSES) {
      store_row(abuf + (buf ^ 1) * MF_A_PASS_U4, pa);
      stage_e(ebuf + (buf ^ 1) * MF_ECOPIES_U32, pd0, pd1);
    }
    __syncthreads();
  }
  // the offset correction of the outputs this wave forms (i below), taken off with P1
  u32 cv[4] = {0u, 0u, 0u, 0u};
  if (sub != 0) {
    const u32* C = mf_corr(Kb, key_off, o) + (sub - 1) * MF_HALF + 128 * wl + n;
#pragma unroll
    for (int nb = 0; nb < 4; nb++) cv[nb] = C[32 * nb];
  }
  // P1 to LDS ([w mod 4][nb][x][lane]); the P2 and P3 waves add it: y0 = P1 + P2 (sub 1,
  // outputs [0, N/2)), y1 = P1 + P3 (sub 2, outputs [N/2, N)).
  u32* p1buf = reinterpret_cast<u32*>(mf_lds);
  if (sub == 0) {
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
#pragma unroll
      for (int x = 0; x < 16; x++) p1buf[((wl * 4 + nb) * 16 + x) * 64 + lane] = (u32)c[nb][x];
  }
  __syncthreads();
  if (sub != 0) {
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
#pragma unroll
      for (int x = 0; x < 16; x++)
        c[nb][x] = (int)((u32)c[nb][x] + p1buf[((wl * 4 + nb) * 16 + x) * 64 + lane] - cv[nb]);
  }
  __syncthreads();
  // y to LDS as rows of MF_PROW words per gate: result (m, i) is lane n + 32 kh, register x of
  // block nb with m = 8 (x / 4) + 4 kh + x % 4, i = (sub - 1) N/2 + 128 (w mod 4) + 32 nb + n
  u32* poly = reinterpret_cast<u32*>(mf_lds);
  if (sub != 0) {
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
#pragma unroll
      for (int x = 0; x < 16; x++)
        poly[(8 * (x >> 2) + 4 * kh + (x & 3)) * MF_PROW + (sub - 1) * MF_HALF + 128 * wl + 32 * nb + n] = (u32)c[nb][x];
  }
  __syncthreads();
  // ACC += y for the gates that bootstrap (coalesced, all loads in flight first); the updated
  // polynomial stays in LDS for the next step's digits. Loads here and below are unconditional,
  // with the gate index clamped into the batch: a guarded load becomes a branch after which the
  // compiler waits for it, one round trip per load.
  {
    constexpr int PER = MF_TILE * RING_N / MF_THREADS + 1;
    u32 av[PER];
    bool lv[PER];
    uint8_t opv[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) opv[q] = 0;
    if (ops) {
#pragma unroll
      for (int q = 0; q < PER; q++) {
        const uint64_t g = mt * MF_TILE + ((tid + q * MF_THREADS) >> 10);
        opv[q] = ops[g < B ? g : 0];
      }
    }
#pragma unroll
    for (int q = 0; q < PER; q++) {
      const int idx = tid + q * MF_THREADS;
      const uint64_t g = mt * MF_TILE + (idx >> 10);
      const uint64_t gc = g < B ? g : 0;
      lv[q] = idx < MF_TILE * RING_N && g < B && op_bootstraps(opv[q]);
      av[q] = acc[(gc * 2 + o) * RING_N + (idx & (RING_N - 1))];
    }
#pragma unroll
    for (int q = 0; q < PER; q++) {
      if (!lv[q]) continue;
      const int idx = tid + q * MF_THREADS, m = idx >> 10, i = idx & (RING_N - 1);
      u32* pp = poly + m * MF_PROW + i;
      const u32 v = av[q] + *pp;
      *pp = v;
      acc[((mt * MF_TILE + m) * 2 + o) * RING_N + i] = v;
    }
  }
  if (next_step < 0) return;
  __syncthreads();
  // Digits of step next_step for rows 3o .. 3o + 2: a 64-lane group per input block kb, lane
  // (m, kh) forming the 16-byte operand of gate m (local coefficients j = 32 kb + 16 kh + 15 - q,
  // q = 0..15, of both halves) for the three levels from the polynomial in LDS, segments 1 and
  // 2 only (the next step forms segment 0 when it stages them); each group writes six 1 KiB
  // operand rows. Gates at or above B and gates that do not bootstrap get zero bytes.
  {
    const int m = lane & 31;
    const uint64_t g = mt * MF_TILE + m;
    const uint64_t gc = g < B ? g : 0;
    const uint8_t op0 = ops ? ops[gc] : (uint8_t)0;
    const bool live = g < B && op_bootstraps(op0);
    const int a = (int)abar[gc * TLWE0 + next_step];
    const u32* pm = poly + m * MF_PROW;
    uint4* dst = reinterpret_cast<uint4*>(Anext + mt * MF_A_TILE + (size_t)GADGET_L * o * MF_A_ROW) + lane;
    for (int kb = wave; kb < MF_KB; kb += MF_WAVES) {
      u32 w[GADGET_L][MF_SUB][4] = {};
      if (live) {
#pragma unroll
        for (int wi = 0; wi < 4; wi++) {
#pragma unroll
          for (int s = 0; s < 4; s++) {
            const int j = 32 * kb + 16 * kh + 15 - 4 * wi - s;
            u32 x[2];
#pragma unroll
            for (int half = 0; half < 2; half++) {
              const int ix = (half * MF_HALF + j - a) & (2 * RING_N - 1);
              const u32 r = pm[ix & (RING_N - 1)];
              x[half] = ((ix & RING_N) ? 0u - r : r) - pm[half * MF_HALF + j] + DECOMP_OFFSET;
            }
#pragma unroll
            for (int k = 0; k < GADGET_L; k++) {
              const int sh = 32 - BG_BIT * (k + 1);
              const u32 d0 = (x[0] >> sh) & 63u, d1 = (x[1] >> sh) & 63u;  // digits plus MF_OFS
              w[k][1][wi] |= (d1 & 255u) << (8 * s);
              w[k][2][wi] |= (d0 & 255u) << (8 * s);
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < GADGET_L; k++)
#pragma unroll
        for (int sg = 1; sg < MF_SUB; sg++)  // segment 0 is formed from these when staged
          dst[((k * MF_SUB + sg) * MF_KB + kb) * 64] = make_uint4(w[k][sg][0], w[k][sg][1], w[k][sg][2], w[k][sg][3]);
    }
  }
}

// Split step for batches too small to fill the chip with (tile, output) workgroups: the work
// of one step is cut into workgroups of four waves per (tile, output o, sub-product s, group
// of TRGSW rows), wave q computing outputs [128 q, 128 q + 128) of P_s over the rows of its
// group and all four byte planes (the pass loop of k_mf_step with one operand segment and one
// key sequence per pass, its products in a diagonal order without the wrap). Each workgroup adds its share of y straight into ACC with
// integer atomic adds (exact in any order: addition mod 2^32): P1 into both halves, P2 into
// y0, P3 into y1. The next step's digits come from a separate launch of k_mf_digits, after
// every share of the step has landed. Row groups: rows [rg * rows, rg * rows + rows) with
// rows = 6 / groups (groups 1, 2, 3 or 6). With groups 12 or 24 every workgroup takes one row
// and a range of 2 or 1 byte planes (planes bhi down to blo): Horner's rule over its own
// planes, then its sum shifted left by 8 blo bits before the atomic add (exact mod 2^32, as
// the full sum is that of the shifted plane sums), so that a single gate spreads over 144
// workgroups.
// With acc_in non-NULL (batches of at most MFP_FUSE gates, one row per workgroup) the step
// needs no digit launch: the accumulator rotates through three buffers, ACC_i in acc_in, the
// target acc zeroed one step earlier, acc_zero (ACC_{i-1}, no longer read) cleared for the
// next step. Each workgroup stages polynomial h of its row r = 3h + k for the batch's gates
// in LDS and forms its own operand segment from it (the digits of X^{abar_i} ACC_h - ACC_h,
// as k_mf_digits would), and the workgroups of sub-products P2 and P3 of the first row group
// also add ACC_i's y0 and y1 halves to their shares, so that acc ends as ACC_{i+1}.
// With part non-NULL (the partial-sum form, any of the counts) the shares are not added but
// stored, P_s of group rg at part[tile][o][s][rg][gate][N/2], and the next digit launch adds
// them into ACC (k_mf_digits with PG = groups). In every form the P2 and P3 workgroups of the
// first group take the operand offset's correction of their outputs off their shares.
// Ek0 (and each tkeys entry) is the start of a whole key; key_off selects the step.
constexpr int MFP_THREADS = 256;
constexpr int MFP_FUSE = 4;  // largest batch whose digits the step kernel forms itself
constexpr int MFP_A_U4 = MF_KB * 64;                                  // one segment of one row: 1024 operands
static_assert(MFP_A_U4 == 4 * MFP_THREADS && MF_S / 4 == MFP_THREADS,
              "four 16-byte operands and one key word per thread and pass");

__global__ __launch_bounds__(MFP_THREADS, 3) void k_mf_part(const int8_t* __restrict__ Ek0, const int8_t* __restrict__ A,
                                                          u32* __restrict__ acc, const uint8_t* __restrict__ ops,
                                                          uint64_t B, int groups,
                                                          const int8_t* const* __restrict__ tkeys, uint64_t key_off,
                                                          const u32* __restrict__ acc_in, u32* __restrict__ acc_zero,
                                                          const u32* __restrict__ abar, int step,
                                                          u32* __restrict__ part) {
  const int8_t* __restrict__ Kb = tkeys ? tkeys[blockIdx.x] : Ek0;
  const int8_t* __restrict__ Ek = Kb + key_off;
  __shared__ uint4 abuf[2][MFP_A_U4];
  __shared__ u32 ebuf[2][4 * MF_COPY_U32];
  const uint64_t mt = blockIdx.x;
  const int o = blockIdx.y;
  const int sub = (int)blockIdx.z % MF_SUB, rg = (int)blockIdx.z / MF_SUB;
  const int rgroups = groups > MF_ROWS ? MF_ROWS : groups;
  const int planes = groups > MF_ROWS ? MF_PLANES * MF_ROWS / groups : MF_PLANES;
  const int rows = MF_ROWS / rgroups, r0 = (rg % rgroups) * rows, passes = planes * rows;
  const int bhi = MF_PLANES - 1 - (rg / rgroups) * planes, blo = bhi - planes + 1;
  const int tid = threadIdx.x, wl = tid >> 6, lane = tid & 63, n = lane & 31, kh = lane >> 5;
  const int tb = MF_HALF + 128 * wl + n - 16 * kh - 15;
  const int cp = tb & 3;
  const int bofs = cp * MF_COPY_U32 + ((tb - cp) >> 2) - 8 * (MF_KB - 1);
  // rotating buffers: the first row group's P2 / P3 workgroups carry ACC_i's y0 / y1 halves
  // into their shares (gates m < MFP_FUSE end in registers x = m of the lanes with kh = 0),
  // fetched here so that their latency hides behind the products
  const bool carry = acc_in != nullptr && rg == 0 && sub != 0;
  u32 cyv[MFP_FUSE][4];
#pragma unroll
  for (int m = 0; m < MFP_FUSE; m++) {
    const uint64_t g = mt * MF_TILE + m;
    const bool fetch = carry && kh == 0 && g < B;
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
      cyv[m][nb] = fetch ? acc_in[(g * 2 + o) * RING_N + (sub == 2 ? MF_HALF : 0) + 128 * wl + 32 * nb + n] : 0u;
  }
  const uint4* Ag = reinterpret_cast<const uint4*>(A + mt * MF_A_TILE) + sub * MFP_A_U4 + tid;
  const u32* Eu = reinterpret_cast<const u32*>(Ek);
  // pass p: plane bhi - p / rows, row r0 + p % rows (any row order gives the same plane sum)
  auto a_row = [&](int pass) { return Ag + (size_t)(r0 + pass % rows) * (MF_A_ROW / 16); };
  auto e_row = [&](int pass) {
    const int r = r0 + pass % rows, b = bhi - pass / rows;
    return Eu + ((((size_t)r * 2 + o) * MF_PLANES + b) * MF_SUB + sub) * (MF_S / 4);
  };
  auto stage_e = [&](u32* dst, u32 d0, u32 d1) {
#pragma unroll
    for (int c = 0; c < 4; c++) dst[c * MF_COPY_U32 + tid] = __builtin_amdgcn_alignbyte(d1, d0, c);
  };
  v16i c[4];
#pragma unroll
  for (int nb = 0; nb < 4; nb++)
#pragma unroll
    for (int x = 0; x < 16; x++) c[nb][x] = 0;
  // one pass: the 16 input blocks of this wave's four output blocks
  auto run_pass = [&](const uint4* Ar, const u32* Bp) {
    auto ldb = [&](int wofs) {
      return v4i{(int)Bp[wofs], (int)Bp[wofs + 1], (int)Bp[wofs + 2], (int)Bp[wofs + 3]};
    };
    auto lda = [](const uint4& u) { return v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w}; };
    // diagonal order without the step kernel's wrap (which needs more registers than this
    // kernel has to spare): group t = 0..18 takes kb = t - 3 + nb for the nb with kb in
    // [0, 16), all with the B operand of diagonal 3 - t, so the key operand stays while the
    // digits change; A blocks are loaded two groups ahead into a ring of eight registers, B
    // operands two groups ahead into a ring of four
    v4i Av[8], Bd[4];
    Av[0] = lda(Ar[0]);
    Av[1] = lda(Ar[64]);
    Bd[0] = ldb(8 * (MF_KB + 2));
    Bd[1] = ldb(8 * (MF_KB + 1));
#pragma unroll
    for (int t = 0; t < MF_KB + 3; t++) {
      if (t + 2 < MF_KB) Av[(t + 2) & 7] = lda(Ar[(t + 2) * 64]);
      if (t + 2 < MF_KB + 3) Bd[(t + 2) & 3] = ldb(8 * (MF_KB - t));
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int nb = 0; nb < 4; nb++) {
        const int kb = t - 3 + nb;
        if (kb >= 0 && kb < MF_KB)
          c[nb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Av[kb & 7], Bd[t & 3], c[nb], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  auto horner_shift = [&]() {
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
#pragma unroll
      for (int x = 0; x < 16; x++) c[nb][x] = (int)((u32)c[nb][x] << 8);
  };
  if (rows == 1) {
    // one TRGSW row: its operands serve all of the workgroup's planes, so they and those
    // planes' key sequences are staged once (the first two in ebuf, the others in the second
    // operand buffer) and the passes run without further loads or barriers
    auto kbuf = [&](int p) -> u32* {
      return p < 2 ? ebuf[p] : reinterpret_cast<u32*>(abuf[1]) + (p - 2) * 4 * MF_COPY_U32;
    };
    const bool fuse = acc_in != nullptr;
    if (!fuse && tid < MF_PLANES * 4 * 4) {  // the tails of all copies of the four key buffers
      const int bufi = tid >> 4, rest = tid & 15;
      kbuf(bufi)[(rest >> 2) * MF_COPY_U32 + MF_S / 4 + (rest & 3)] = 0u;
    }
    uint4 x0 = make_uint4(0u, 0u, 0u, 0u), x1 = x0, x2 = x0, x3 = x0;
    if (!fuse) {
      const uint4* as = a_row(0);
      x0 = as[0];
      x1 = as[MFP_THREADS];
      x2 = as[2 * MFP_THREADS];
      x3 = as[3 * MFP_THREADS];
    }
    u32 d0[MF_PLANES], d1[MF_PLANES];
#pragma unroll
    for (int p = 0; p < MF_PLANES; p++) {
      d0[p] = d1[p] = 0u;
      if (p < planes) {  // uniform
        const u32* er = e_row(p);
        d0[p] = er[tid];
        d1[p] = (tid + 1 < MF_S / 4) ? er[tid + 1] : 0u;
      }
    }
    if (fuse) {
      // this row's operand segment from ACC_i: stage polynomial h of the gates in LDS (the
      // second operand buffer), zero the operands of gates without digits, then form the
      // digit words of the others (gate m, block kb, half kh, word wi: four coefficients)
      const int h = r0 / GADGET_L, k = r0 % GADGET_L, sh = 32 - BG_BIT * (k + 1);
      const uint64_t g0 = mt * MF_TILE;
      const int nb = (int)((B - g0 < (uint64_t)MFP_FUSE) ? B - g0 : (uint64_t)MFP_FUSE);
      u32* pst = reinterpret_cast<u32*>(abuf[1]);  // [MFP_FUSE][N]
      bool gl[MFP_FUSE];
      uint4 pv[MFP_FUSE];
#pragma unroll
      for (int m = 0; m < MFP_FUSE; m++) {
        gl[m] = m < nb && (!ops || op_bootstraps(ops[g0 + m]));
        pv[m] = gl[m] ? reinterpret_cast<const uint4*>(acc_in + ((g0 + m) * 2 + h) * RING_N)[tid]
                      : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int m = 0; m < MFP_FUSE; m++) reinterpret_cast<uint4*>(pst + m * RING_N)[tid] = pv[m];
      __syncthreads();
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int c = tid + MFP_THREADS * v, m = c & 31;
        if (!(m < MFP_FUSE && gl[m])) abuf[0][c] = make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int v = 0; v < 2; v++) {
        const int u = tid + MFP_THREADS * v, m = u >> 7, kb = (u >> 3) & 15, kq = (u >> 2) & 1, wi = u & 3;
        if (!gl[m]) continue;
        const u32* P = pst + m * RING_N;
        const int a = (int)abar[(g0 + m) * TLWE0 + step];
        u32 w = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {  // byte q of the word: local coefficient j
          const int j = 32 * kb + 16 * kq + 15 - 4 * wi - q;
          u32 d[2];
#pragma unroll
          for (int half = 0; half < 2; half++) {
            const int ix = (half * MF_HALF + j - a) & (2 * RING_N - 1);
            const u32 r = P[ix & (RING_N - 1)];
            const u32 x = ((ix & RING_N) ? 0u - r : r) - P[half * MF_HALF + j] + DECOMP_OFFSET;
            d[half] = (x >> sh) & 63u;  // digit plus MF_OFS
          }
          const u32 byte = sub == 0 ? d[0] + d[1] : (sub == 1 ? d[1] : d[0]);
          w |= (byte & 255u) << (8 * q);
        }
        reinterpret_cast<u32*>(&abuf[0][kb * 64 + m + 32 * kq])[wi] = w;
      }
      __syncthreads();  // the staged polynomials are read; the key buffers may now use abuf[1]
      if (tid < MF_PLANES * 4 * 4) {
        const int bufi = tid >> 4, rest = tid & 15;
        kbuf(bufi)[(rest >> 2) * MF_COPY_U32 + MF_S / 4 + (rest & 3)] = 0u;
      }
    } else {
      abuf[0][tid] = x0;
      abuf[0][tid + MFP_THREADS] = x1;
      abuf[0][tid + 2 * MFP_THREADS] = x2;
      abuf[0][tid + 3 * MFP_THREADS] = x3;
    }
#pragma unroll
    for (int p = 0; p < MF_PLANES; p++)
      if (p < planes) stage_e(kbuf(p), d0[p], d1[p]);
    __syncthreads();
#pragma unroll 1
    for (int pass = 0; pass < planes; pass++) {
      run_pass(abuf[0] + lane, kbuf(pass) + bofs);
      if (pass + 1 < planes) horner_shift();
    }
  } else {
    if (tid < 2 * 4 * 4) {  // the tails of all copies of both buffers
      const int bufi = tid >> 4, rest = tid & 15;
      ebuf[bufi][(rest >> 2) * MF_COPY_U32 + MF_S / 4 + (rest & 3)] = 0u;
    }
    {
      const uint4* as = a_row(0);
      const uint4 x0 = as[0], x1 = as[MFP_THREADS], x2 = as[2 * MFP_THREADS], x3 = as[3 * MFP_THREADS];
      const u32* er = e_row(0);
      const u32 d0 = er[tid], d1 = (tid + 1 < MF_S / 4) ? er[tid + 1] : 0u;
      abuf[0][tid] = x0;
      abuf[0][tid + MFP_THREADS] = x1;
      abuf[0][tid + 2 * MFP_THREADS] = x2;
      abuf[0][tid + 3 * MFP_THREADS] = x3;
      stage_e(ebuf[0], d0, d1);
    }
    __syncthreads();
    for (int pass = 0; pass < passes; pass++) {
      const int buf = pass & 1;
      const int nx = (pass + 1 < passes) ? pass + 1 : pass;  // the last pass fetches itself again, unused
      const uint4* as = a_row(nx);
      const uint4 p0 = as[0], p1 = as[MFP_THREADS], p2 = as[2 * MFP_THREADS], p3 = as[3 * MFP_THREADS];
      u32 pd0, pd1;
      {
        const u32* er = e_row(nx);
        pd0 = er[tid];
        pd1 = (tid + 1 < MF_S / 4) ? er[tid + 1] : 0u;
      }
      run_pass(abuf[buf] + lane, ebuf[buf] + bofs);
      if (pass % rows == rows - 1 && pass + 1 < passes) horner_shift();
      if (pass + 1 < passes) {
        uint4* ad = abuf[buf ^ 1] + tid;
        ad[0] = p0;
        ad[MFP_THREADS] = p1;
        ad[2 * MFP_THREADS] = p2;
        ad[3 * MFP_THREADS] = p3;
        stage_e(ebuf[buf ^ 1], pd0, pd1);
      }
      __syncthreads();
    }
  }
  // the first group's P2 / P3 workgroups also take the offset correction of their outputs off
  u32 cv[4] = {0u, 0u, 0u, 0u};
  if (rg == 0 && sub != 0) {
    const u32* C = mf_corr(Kb, key_off, o) + (sub - 1) * MF_HALF + 128 * wl + n;
#pragma unroll
    for (int nb = 0; nb < 4; nb++) cv[nb] = C[32 * nb];
  }
  // gates of the tile that bootstrap: bit m of `live` (lanes 0..31 test gate m = lane)
  bool mine = false;
  {
    const uint64_t g = mt * MF_TILE + n;
    const uint8_t op = ops ? ops[g < B ? g : 0] : (uint8_t)0;
    mine = kh == 0 && g < B && op_bootstraps(op);
  }
  const uint64_t live = __ballot(mine);
  // rotating buffers: the first row group's P1 workgroup clears the next step's target
  if (acc_in != nullptr && rg == 0 && sub == 0) {  // rows of gates that do not bootstrap stay untouched
    for (int m = 0; m < MFP_FUSE; m++)
      if ((live >> m) & 1)
        reinterpret_cast<uint4*>(acc_zero + ((mt * MF_TILE + m) * 2 + o) * RING_N)[tid] = make_uint4(0u, 0u, 0u, 0u);
  }
  // result (m, i): lane n + 32 kh, register x of block nb, m = 8 (x / 4) + 4 kh + x % 4,
  // i = 128 q + 32 nb + n; P1 adds into outputs i and N/2 + i, P2 into i, P3 into N/2 + i
  if (part) {  // partial-sum form: plain stores of the share, added up by the digit launch
    u32* q = part + (((mt * 2 + o) * MF_SUB + sub) * (uint64_t)groups + rg) * MF_PART_U32 + 128 * wl + n;
#pragma unroll
    for (int x = 0; x < 16; x++) {
      const int m = 8 * (x >> 2) + 4 * kh + (x & 3);
      if (!((live >> m) & 1)) continue;
#pragma unroll
      for (int nb = 0; nb < 4; nb++) q[(size_t)m * MF_HALF + 32 * nb] = ((u32)c[nb][x] << (8 * blo)) - cv[nb];
    }
    return;
  }
#pragma unroll
  for (int x = 0; x < 16; x++) {
    const int m = 8 * (x >> 2) + 4 * kh + (x & 3);
    if (!((live >> m) & 1)) continue;
    u32* row = acc + ((mt * MF_TILE + m) * 2 + o) * RING_N + 128 * wl + n;
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      const u32 v = ((u32)c[nb][x] << (8 * blo)) - cv[nb];
      const u32 cy = (x < MFP_FUSE && carry) ? cyv[x < MFP_FUSE ? x : 0][nb] : 0u;
      if (sub != 2) atomicAdd(row + 32 * nb, v + cy);
      if (sub != 1) atomicAdd(row + MF_HALF + 32 * nb, v + cy);
    }
  }
}

hipError_t init_mf_kernel_attributes() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_step), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)MF_STEP_LDS);
}

size_t mf_key_bytes() { return MF_KEY_BYTES + (size_t)LWE_N * MF_CORR_STEP_U32 * 4; }

size_t mf_work_bytes(uint64_t B, bool need_acc) {
  const uint64_t tiles = (B + MF_TILE - 1) / MF_TILE;
  const uint64_t ptiles = tiles < (uint64_t)kPartTiles ? tiles : (uint64_t)kPartTiles;
  const uint64_t stiles = tiles < (uint64_t)kPartSmallTiles ? tiles : (uint64_t)kPartSmallTiles;
  const uint64_t blocks = std::max<uint64_t>(ptiles * 6, stiles * 24);  // share blocks per (output, sub-product)
  return 2 * tiles * MF_A_TILE + (need_acc ? (size_t)B * 2 * RING_N * 4 : 0) +
         (size_t)blocks * 2 * MF_SUB * MF_PART_U32 * 4;
}

hipError_t launch_mf_key(const uint32_t* bk, int8_t* E, hipStream_t st) {
  const uint64_t rows = (uint64_t)LWE_N * MF_ROWS * 2;
  hipLaunchKernelGGL(k_mf_key, dim3((unsigned)((rows * MF_S + 255) / 256)), dim3(256), 0, st, bk, E, rows);
  hipLaunchKernelGGL(k_mf_corr, dim3((unsigned)LWE_N, 2), dim3(256), 0, st, bk,
                     reinterpret_cast<u32*>(E + MF_KEY_BYTES));
  return hipGetLastError();
}

hipError_t launch_blind_rotate_mfma(const vsp_context* ctx, const uint8_t* ops, const uint32_t* abar, uint32_t* tlwe1,
                                    uint32_t* trlwe, uint64_t B, void* work, hipStream_t st, bool instrument,
                                    const int8_t* const* tkeys) {
  if (B == 0) return hipSuccess;
  const uint64_t tiles = (B + MF_TILE - 1) / MF_TILE;
  // operands of even steps in A[0], of odd steps in A[1]: step i reads A[i % 2] and writes
  // the operands of step i + 1 into the other one
  int8_t* Ab[2] = {static_cast<int8_t*>(work), static_cast<int8_t*>(work) + tiles * MF_A_TILE};
  u32* acc = trlwe ? trlwe : reinterpret_cast<u32*>(Ab[1] + tiles * MF_A_TILE);
  hipLaunchKernelGGL(k_mf_init, dim3((unsigned)((B * 2 * RING_N + 255) / 256)), dim3(256), 0, st, ops, abar, acc, B,
                     nullptr);
  hipLaunchKernelGGL(k_mf_digits<0>, dim3((unsigned)tiles, 2, MF_TILE / MF_DG), dim3(256), 0, st, ops, abar, acc, Ab[0],
                     B, 0, nullptr);
  {
    // one event pair around the whole step sequence: its duration / LWE_N is the average step
    // launch including the gaps between launches (an upper bound on the kernel's own time)
    ProfScope ps(instrument ? ctx : nullptr, 3, st, LWE_N);
    for (int i = 0; i < LWE_N; i++)
      hipLaunchKernelGGL(k_mf_step, dim3((unsigned)tiles, 2), dim3(MF_THREADS), MF_STEP_LDS, st,
                         tkeys ? nullptr : ctx->mf_key, Ab[i & 1], acc, ops, B,
                         Ab[(i + 1) & 1], abar, i + 1 < LWE_N ? i + 1 : -1, tkeys, (uint64_t)i * MF_KEY_STEP);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && tlwe1) e = launch_sample_extract(acc, tlwe1, B, 1, st);
  return e;
}

// Split form of the matrix-core blind rotation: per step one k_mf_part launch (shares of the
// products added into ACC) and one k_mf_digits launch (the next step's operands from ACC).
// groups (kSplitGroupChoices) sets the TRGSW rows, or for one row the byte planes, per
// workgroup; a negative count -g (g = 1, 2, 3, 6, or 12 and 24 for at most eight tiles) stores
// the shares as partial sums that the digit launch adds up, instead of integer atomics. The workspace is mf_work_bytes(B, .):
// the operands of one step, without a caller TRLWE the accumulators, then the partial sums.
template <int PG>
static void launch_split_partial_steps(const vsp_context* ctx, const uint8_t* ops, const uint32_t* abar, u32* acc,
                                       int8_t* Aop, u32* Q, uint64_t B, uint64_t tiles, hipStream_t st,
                                       bool instrument, const int8_t* const* tkeys) {
  const dim3 dgrid((unsigned)tiles, 2, MF_TILE / MF_DG), pgrid((unsigned)tiles, 2, (unsigned)(MF_SUB * PG));
  constexpr int DG = 2;
  const dim3 rgrid((unsigned)tiles, 2, MF_TILE / DG);
  hipLaunchKernelGGL(k_mf_digits<0>, dgrid, dim3(256), 0, st, ops, abar, acc, Aop, B, 0, nullptr);
  ProfScope ps(instrument ? ctx : nullptr, 3, st, LWE_N);
  for (int i = 0; i < LWE_N; i++) {
    hipLaunchKernelGGL(k_mf_part, pgrid, dim3(MFP_THREADS), 0, st,
                       tkeys ? nullptr : ctx->mf_key, Aop, acc, ops, B, PG, tkeys,
                       (uint64_t)i * MF_KEY_STEP, nullptr, nullptr, nullptr, 0, Q);
    hipLaunchKernelGGL((k_mf_digits<PG, DG>), rgrid, dim3(256), 0, st, ops, abar, acc, Aop, B, i + 1, Q);
  }
}

hipError_t launch_blind_rotate_mfsplit(const vsp_context* ctx, const uint8_t* ops, const uint32_t* abar,
                                       uint32_t* tlwe1, uint32_t* trlwe, uint64_t B, void* work, int groups,
                                       hipStream_t st, bool instrument, const int8_t* const* tkeys) {
  if (B == 0) return hipSuccess;
  if (!split_groups_valid(groups)) return hipErrorInvalidValue;
  const uint64_t tiles = (B + MF_TILE - 1) / MF_TILE;
  if (groups < 0 && tiles > (uint64_t)(groups < -6 ? kPartSmallTiles : kPartTiles))
    groups = -groups;  // no room for the partial sums
  int8_t* Aop = static_cast<int8_t*>(work);
  u32* acc = trlwe ? trlwe : reinterpret_cast<u32*>(Aop + 2 * tiles * MF_A_TILE);
  u32* Q = reinterpret_cast<u32*>(Aop + 2 * tiles * MF_A_TILE + (trlwe ? 0 : B * 2 * RING_N * 4));
  if (groups < 0) {
    hipLaunchKernelGGL(k_mf_init, dim3((unsigned)((B * 2 * RING_N + 255) / 256)), dim3(256), 0, st, ops, abar, acc, B,
                       nullptr);
    switch (-groups) {
      case 1: launch_split_partial_steps<1>(ctx, ops, abar, acc, Aop, Q, B, tiles, st, instrument, tkeys); break;
      case 2: launch_split_partial_steps<2>(ctx, ops, abar, acc, Aop, Q, B, tiles, st, instrument, tkeys); break;
      case 3: launch_split_partial_steps<3>(ctx, ops, abar, acc, Aop, Q, B, tiles, st, instrument, tkeys); break;
      case 6: launch_split_partial_steps<6>(ctx, ops, abar, acc, Aop, Q, B, tiles, st, instrument, tkeys); break;
      case 12: launch_split_partial_steps<12>(ctx, ops, abar, acc, Aop, Q, B, tiles, st, instrument, tkeys); break;
      default: launch_split_partial_steps<24>(ctx, ops, abar, acc, Aop, Q, B, tiles, st, instrument, tkeys); break;
    }
  } else if (B <= (uint64_t)MFP_FUSE && groups >= MF_ROWS) {
    // one launch per step: ACC_i in buf[i mod 3], the step adds into buf[(i + 1) mod 3] and
    // clears buf[(i + 2) mod 3]; n is a multiple of 3, so ACC_n ends in buf[0] = acc. The
    // two spare buffers take the (unused) operand area of the workspace.
    static_assert(LWE_N % 3 == 0, "the last step's target is the first buffer");
    static_assert(2 * MFP_FUSE * 2 * RING_N * 4 <= 2 * MF_A_TILE, "spare buffers fit the operand area");
    const dim3 pgrid((unsigned)tiles, 2, (unsigned)(MF_SUB * groups));
    u32* buf[3] = {acc, reinterpret_cast<u32*>(Aop), reinterpret_cast<u32*>(Aop) + B * 2 * RING_N};
    hipLaunchKernelGGL(k_mf_init, dim3((unsigned)((B * 2 * RING_N + 255) / 256)), dim3(256), 0, st, ops, abar, acc, B,
                       buf[1]);
    ProfScope ps(instrument ? ctx : nullptr, 3, st, LWE_N);
    for (int i = 0; i < LWE_N; i++)
      hipLaunchKernelGGL(k_mf_part, pgrid, dim3(MFP_THREADS), 0, st,
                         tkeys ? nullptr : ctx->mf_key, Aop, buf[(i + 1) % 3], ops, B,
                         groups, tkeys, (uint64_t)i * MF_KEY_STEP, buf[i % 3], buf[(i + 2) % 3], abar, i, nullptr);
  } else {
    constexpr int DG = 2;
    const dim3 dgrid((unsigned)tiles, 2, MF_TILE / DG), pgrid((unsigned)tiles, 2, (unsigned)(MF_SUB * groups));
    hipLaunchKernelGGL(k_mf_init, dim3((unsigned)((B * 2 * RING_N + 255) / 256)), dim3(256), 0, st, ops, abar, acc, B,
                       nullptr);
    hipLaunchKernelGGL((k_mf_digits<0, DG>), dgrid, dim3(256), 0, st, ops, abar, acc, Aop, B, 0, nullptr);
    ProfScope ps(instrument ? ctx : nullptr, 3, st, LWE_N);
    for (int i = 0; i < LWE_N; i++) {
      hipLaunchKernelGGL(k_mf_part, pgrid, dim3(MFP_THREADS), 0, st,
                         tkeys ? nullptr : ctx->mf_key, Aop, acc, ops, B, groups, tkeys,
                         (uint64_t)i * MF_KEY_STEP, nullptr, nullptr, nullptr, 0, nullptr);
      if (i + 1 < LWE_N)
        hipLaunchKernelGGL((k_mf_digits<0, DG>), dgrid, dim3(256), 0, st, ops, abar, acc, Aop, B, i + 1, nullptr);
    }
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && tlwe1) e = launch_sample_extract(acc, tlwe1, B, 1, st);
  return e;
}

}  // namespace vsp
