// Wave-level negacyclic NTT of degree N = 1024 modulo p = 2^64 - 2^32 + 1, and the TRGSW x
// TRLWE external product built on it (Sec. 2.1.2, TRGSW and CMUX).
//
// Layout. A wave (64 lanes) works on two polynomials at once: lanes 0-31 on the first,
// lanes 32-63 on the second. Lane l = lane & 31 holds coefficients l + 32 t (t = 0..31) in
// register t. With Z = X^32 the polynomial is sum_l X^l (sum_t a_{l+32t} Z^t), so:
//  pass 1 (in registers): for every l, the 32-point negacyclic transform over t evaluates
//    sum_t a_{l+32t} zeta^t at the 32 roots zeta = 2^{3(2u+1)} of Z^32 = -1, giving the
//    residues a mod (X^32 - zeta_u). Its twiddles are powers of two (2 has order 192 mod p),
//    so every multiply is by a compile-time 2^e.
//  transpose through LDS: lane u receives the 32 coefficients of residue u.
//  pass 2 (in registers): a mod (X^32 - zeta_u) is evaluated at psi_u w^k (w = 2^6, a
//    primitive 32nd root; psi_u = psi^{2u+1} with psi^32 = 8): multiply coefficient j by
//    psi_u^j (table) then a cyclic 32-point DFT with power-of-two twiddles.
// The inverse undoes pass 2 (inverse DFT, psi_u^-j), transposes back, and undoes pass 1 as
// a cyclic inverse DFT over the residues followed by the twist zeta^-t of coefficient t.
// The factor 1/N is folded into the key. Every butterfly multiplies its second input by the
// twiddle (Cooley-Tukey form), so the product is canonical and the sum and difference
// need a single carry fix each.
#pragma once
#include "gl64.h"

namespace vsp {

constexpr int RING_N = 1024;
constexpr int LWE_N = 630;
constexpr int GADGET_L = 3;
constexpr int BG_BIT = 6;
constexpr int KS_T = 8;
constexpr int KS_BASEBIT = 2;
constexpr u32 MU = 1u << 29;                // 1/8
constexpr u32 DECOMP_OFFSET = 0x82082000u;  // sum_r (Bg/2) 2^(32-6r) + 2^(32-18-1)

// One transpose region per half-wave: 32 rows of 33 u32 (the pad column keeps the row and
// column accesses of a half-wave on distinct LDS banks); 64-bit values cross it in two
// 32-bit passes. The regions of the two halves start 32 words apart modulo the bank count.
constexpr int TROW = 33;
constexpr int TREGION = 32 * TROW + 64;     // u32 per half
constexpr int WAVE_T_U32 = 2 * TREGION;     // u32 per wave

// External-product key layout in u64, per TRGSW: [round k][slot s][lane][e]: lane l + 32 h
// holds, for output polynomial h (0: a, 1: b), entry e = 0 from TRGSW row k (the row that
// multiplies the digits of ACC.a) and e = 1 from row k + 3 (digits of ACC.b). One 16-byte
// load gives a lane both entries of a slot.
constexpr int TRGSW_NTT_U64 = GADGET_L * 32 * 64 * 2;

constexpr int brv5(int k) {
  return ((k & 1) << 4) | ((k & 2) << 2) | (k & 4) | ((k & 8) >> 2) | ((k & 16) >> 4);
}

// Twiddle exponents: every twiddle of the two in-register passes is 2^e mod p, e in [0, 192).
struct TwiddleExps {
  int p1f[32];   // pass-1 forward: 3 brv5(m)
  int p1i[32];   // pass-1 inverse: -3 brv5(m)
  int dft[32];   // w^e = 2^{6e}
  int dfti[32];  // w^-e
};

constexpr TwiddleExps make_twiddle_exps() {
  TwiddleExps T{};
  for (int m = 0; m < 32; m++) {
    T.p1f[m] = (3 * brv5(m)) % 192;
    T.p1i[m] = (192 - 3 * brv5(m)) % 192;
    T.dft[m] = (6 * m) % 192;
    T.dfti[m] = (192 - 6 * m) % 192;
  }
  return T;
}

__device__ constexpr TwiddleExps kTwE = make_twiddle_exps();

// Cooley-Tukey butterfly (x, y) -> (x + 2^E y, x - 2^E y), E in [0, 192); 2^96 = -1 folds
// the upper half of the exponents into a swap of the sum and the difference.
__device__ __forceinline__ void bfly_ct(u64& x, u64& y, int E) {
  const u64 a = x;
  const u64 t = gl_mul_pow2(y, E % 96);  // canonical
  if (E >= 96) {
    x = gl_sub_c(a, t);
    y = gl_add_c(a, t);
  } else {
    x = gl_add_c(a, t);
    y = gl_sub_c(a, t);
  }
}

// Hides x from the optimiser so that per-lane address arithmetic derived from it is
// recomputed inside a loop instead of being hoisted (and kept live) across all iterations.
__device__ __forceinline__ int opaque_lane(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Orders the LDS traffic of one wave (all lanes' stores before any lane's loads).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pass 1, forward: negacyclic Cooley-Tukey over the register index (natural order in,
// bit-reversed out: register k holds residue u = brv5(k)). With SMALL the inputs are signed
// integers of at most 2^6 in magnitude (two's complement in the 64-bit word), and the first
// stage, x +- 2^48 y, is computed exactly in 64-bit integers before entering the field.
template <bool SMALL>
__device__ __forceinline__ void pass1_forward(u64 (&v)[32]) {
  static_assert(3 * 16 == 48, "first-stage twiddle zeta^16 = 2^48");
#pragma unroll
  for (int s = 0; s < 5; s++) {
    const int M = 1 << s, H = 16 >> s;
#pragma unroll
    for (int b = 0; b < M; b++) {
#pragma unroll
      for (int j = 0; j < H; j++) {
        const int i = b * 2 * H + j;
        if (SMALL && s == 0) {
          const int64_t x = (int64_t)v[i], y = (int64_t)v[i + H] * ((int64_t)1 << 48);
          const int64_t sp = x + y, sm = x - y;  // |.| < 2^54
          v[i] = (u64)sp - ((sp < 0) ? GL_EPS : 0);
          v[i + H] = (u64)sm - ((sm < 0) ? GL_EPS : 0);
        } else {
          bfly_ct(v[i], v[i + H], kTwE.p1f[M + b]);
        }
      }
    }
  }
}

// Cyclic 32-point DFT with w = 2^6 (natural order in, bit-reversed out: register brv5(k)
// receives X_k), as decimation in time over the bit-reversed register names.
__device__ __forceinline__ void dft32_forward(u64 (&v)[32]) {
#pragma unroll
  for (int s = 4; s >= 0; s--) {
    const int H = 16 >> s;
#pragma unroll
    for (int blk = 0; blk < 32; blk += 2 * H) {
#pragma unroll
      for (int j = 0; j < H; j++) bfly_ct(v[brv5(blk + j)], v[brv5(blk + j + H)], kTwE.dft[(j << s) & 31]);
    }
  }
}

// Cyclic inverse DFT with w^-1 (decimation in time; bit-reversed in, natural out; unscaled).
// Inverts dft32_forward, and also pass 1: register k of a lane holding the residues at
// zeta w^brv5(k) yields sum_u A_u w^-ut in register t.
__device__ __forceinline__ void dft32_inverse(u64 (&v)[32]) {
#pragma unroll
  for (int s = 4; s >= 0; s--) {
    const int H = 16 >> s;
#pragma unroll
    for (int blk = 0; blk < 32; blk += 2 * H) {
#pragma unroll
      for (int j = 0; j < H; j++) bfly_ct(v[blk + j], v[blk + j + H], kTwE.dfti[(j << s) & 31]);
    }
  }
}

// Lane l, register k (residue brv5(k), coefficient l) -> lane u = brv5(k), register l,
// through the half-wave's u32 region (low words, then high words).
__device__ __forceinline__ void transpose_forward(u64 (&v)[32], u32* reg, int l) {
  u32 lo[32];
#pragma unroll
  for (int k = 0; k < 32; k++) reg[brv5(k) * TROW + l] = (u32)v[k];
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < 32; j++) lo[j] = reg[l * TROW + j];
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < 32; k++) reg[brv5(k) * TROW + l] = (u32)(v[k] >> 32);
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < 32; j++) v[j] = ((u64)reg[l * TROW + j] << 32) | lo[j];
  wave_lds_sync();
}

// Inverse of transpose_forward.
__device__ __forceinline__ void transpose_inverse(u64 (&v)[32], u32* reg, int l) {
  u32 lo[32];
#pragma unroll
  for (int j = 0; j < 32; j++) reg[j * TROW + l] = (u32)v[j];
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < 32; k++) lo[k] = reg[l * TROW + brv5(k)];
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < 32; j++) reg[j * TROW + l] = (u32)(v[j] >> 32);
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < 32; k++) v[k] = ((u64)reg[l * TROW + brv5(k)] << 32) | lo[k];
  wave_lds_sync();
}

// v[j] *= T[j][l] for j >= 1 (T[0][*] = 1), loading the table entries eight at a time so that
// at most sixteen of them are in flight.
__device__ __forceinline__ void table_multiply(u64 (&v)[32], const u64* T, int l) {
#pragma unroll
  for (int c = 0; c < 4; c++) {
    u64 w[8];
#pragma unroll
    for (int q = 0; q < 8; q++) w[q] = (8 * c + q == 0) ? 1 : T[(8 * c + q) * 32 + l];
#pragma unroll
    for (int q = 0; q < 8; q++)
      if (8 * c + q != 0) v[8 * c + q] = gl_mul(v[8 * c + q], w[q]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Forward transform of this half's polynomial (values already residues mod p; with SMALL,
// signed integers of magnitude at most 2^6). tf is the [j][u] table psi_u^j (in LDS or
// global memory).
template <bool SMALL = false>
__device__ __forceinline__ void ntt_forward(u64 (&v)[32], const u64* tf, u32* reg, int l) {
  pass1_forward<SMALL>(v);
  transpose_forward(v, reg, l);
  table_multiply(v, tf, l);
  dft32_forward(v);
}

// Inverse transform, lifted: out[t] receives coefficient l + 32 t of N times the polynomial,
// as the exact integer in (-p/2, p/2) reduced mod 2^32 (ti is psi_u^-j). After the inverse
// DFT over the residues, coefficient t still carries zeta^t; zeta^-t = 2^(192 - 3t) =
// -2^(96 - 3t) removes it, the sign going into the final negation.
__device__ __forceinline__ void ntt_inverse_lift(u64 (&v)[32], const u64* ti, u32* reg, int l, u32 (&out)[32]) {
  dft32_inverse(v);
  table_multiply(v, ti, l);
  transpose_inverse(v, reg, l);
  dft32_inverse(v);
  out[0] = gl_lift_u32(gl_canon(v[0]));
#pragma unroll
  for (int t = 1; t < 32; t++) out[t] = 0u - gl_lift_u32(gl_mul_pow2(v[t], 96 - 3 * t));
}

// Gadget digit of a torus value at bit offset sh = 32 - 6r (r = 1..3): signed in [-32, 31],
// returned sign-extended to 64 bits (the small-input form of ntt_forward). The rounding
// offset makes the l digits a round-to-nearest decomposition.
__device__ __forceinline__ u64 gadget_digit(u32 x, int sh) {
  const u32 t = x + DECOMP_OFFSET;
  return (u64)(int64_t)((int32_t)((t >> sh) & 63u) - 32);
}

// Both halves' values of one slot: v_permlane32_swap(x, x) exchanges the upper half-wave of
// its first operand with the lower half-wave of its second, so afterwards the first result
// holds the lanes 0-31 value (the digit transform of ACC.a) and the second the lanes 32-63
// value (ACC.b) in every lane.
__device__ __forceinline__ void both_halves(u64 x, u64& xa, u64& xb) {
  const auto lo = __builtin_amdgcn_permlane32_swap((u32)x, (u32)x, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((u32)(x >> 32), (u32)(x >> 32), false, false);
  xa = ((u64)hi[0] << 32) | lo[0];
  xb = ((u64)hi[1] << 32) | lo[1];
}

// Wave-cooperative external product: out = this half's polynomial of C (ext) D (lifted to
// the torus). D holds this half's polynomial of the TRLWE operand (lanes 0-31: a, lanes
// 32-63: b); Cn is the TRGSW in the key layout above (already scaled by 1/N). Round k
// transforms gadget digit k+1 of both halves (TRGSW rows k and k+3); each lane takes both
// halves' transformed digits of a slot and adds their products with its output polynomial's
// two key entries to its accumulator, reducing the 129-bit sum once. Key entries stream in
// chunks of KCH slots, the next chunk in flight while the current one is used.
constexpr int KCH = 4;

// DigitSource: callable (int sh, u64 (&x)[32]) filling x with the gadget digit at bit offset
// sh of this half's operand polynomial (as residues), e.g. OperandDigits below.
template <class DigitSource>
__device__ __forceinline__ void external_product(DigitSource digits, const u64* __restrict__ Cn, const u64* tf,
                                                 const u64* ti, u32* reg, int lane, u32 (&out)[32]) {
  const int l = lane & 31;
  u64 x[32], sum[32];
#pragma unroll
  for (int s = 0; s < 32; s++) sum[s] = 0;
#pragma unroll 1
  for (int k = 0; k < GADGET_L; k++) {
    const ulonglong2* key = reinterpret_cast<const ulonglong2*>(Cn) + (size_t)k * 32 * 64 + lane;
    ulonglong2 kc[KCH];
#pragma unroll
    for (int q = 0; q < KCH; q++) kc[q] = key[q * 64];
    digits(32 - BG_BIT * (k + 1), x);
    ntt_forward<true>(x, tf, reg, l);
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
  ntt_inverse_lift(sum, ti, reg, l, out);
}

// Digits of an operand polynomial held in registers.
struct OperandDigits {
  const u32 (&D)[32];
  __device__ __forceinline__ void operator()(int sh, u64 (&x)[32]) const {
#pragma unroll
    for (int t = 0; t < 32; t++) x[t] = gadget_digit(D[t], sh);
  }
};

// Coefficient j of X^k * (mu, mu, ..., mu), k in [0, 2N).
__device__ __forceinline__ u32 rotated_testvector(int j, int k) {
  const bool wrap = j < (k & (RING_N - 1));
  const bool neg = wrap != (k >= RING_N);
  return neg ? (0u - MU) : MU;
}

// D = X^k * P - P for this half's polynomial (k in [0, 2N)), through the LDS region.
__device__ __forceinline__ void rotate_minus(const u32 (&P)[32], int k, u32* buf, int l, u32 (&D)[32]) {
#pragma unroll
  for (int t = 0; t < 32; t++) buf[l + 32 * t] = P[t];
  wave_lds_sync();
#pragma unroll
  for (int t = 0; t < 32; t++) {
    const int idx = (l + 32 * t - k) & (2 * RING_N - 1);
    u32 v = buf[idx & (RING_N - 1)];
    if (idx & RING_N) v = 0u - v;
    D[t] = v - P[t];
  }
  wave_lds_sync();
}

}  // namespace vsp
