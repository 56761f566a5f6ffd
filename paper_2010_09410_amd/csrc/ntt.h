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
// The inverse runs the same steps backwards; the factor 1/N is folded into the key.
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

// One transform region: 32 rows of 33 u64 (the pad column keeps LDS accesses conflict-free).
constexpr int TROW = 33;
constexpr int TREGION = 32 * TROW + 16;     // + pad so the two halves start 16 u64 apart
constexpr int WAVE_LDS_U64 = 2 * TREGION;   // per wave

// External-product key layout in u64: [round k][c'][slot s][lane] per TRGSW, where
// lanes 0-31 carry row k and lanes 32-63 row k+3; c' = 0 is the output polynomial the
// half owns (a for lanes 0-31, b for lanes 32-63) and c' = 1 the other one.
constexpr int TRGSW_NTT_U64 = GADGET_L * 2 * 32 * 64;

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
  if (E >= 96) {
    const u64 t = gl_mul_pow2(y, E - 96);
    x = gl_sub(a, t);
    y = gl_add(a, t);
  } else {
    const u64 t = gl_mul_pow2(y, E);
    x = gl_add(a, t);
    y = gl_sub(a, t);
  }
}

// Gentleman-Sande butterfly (x, y) -> (x + y, (x - y) 2^E), E in [0, 192).
__device__ __forceinline__ void bfly_gs(u64& x, u64& y, int E) {
  const u64 a = x, b = y;
  x = gl_add(a, b);
  y = (E >= 96) ? gl_mul_pow2(gl_sub(b, a), E - 96) : gl_mul_pow2(gl_sub(a, b), E);
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
// bit-reversed out: register k holds residue u = brv5(k)).
__device__ __forceinline__ void pass1_forward(u64 (&v)[32]) {
#pragma unroll
  for (int s = 0; s < 5; s++) {
    const int M = 1 << s, H = 16 >> s;
#pragma unroll
    for (int b = 0; b < M; b++) {
#pragma unroll
      for (int j = 0; j < H; j++) {
        const int i = b * 2 * H + j;
        bfly_ct(v[i], v[i + H], kTwE.p1f[M + b]);
      }
    }
  }
}

// Pass 1, inverse (Gentleman-Sande; bit-reversed in, natural out; unscaled).
__device__ __forceinline__ void pass1_inverse(u64 (&v)[32]) {
#pragma unroll
  for (int s = 4; s >= 0; s--) {
    const int M = 1 << s, H = 16 >> s;
#pragma unroll
    for (int b = 0; b < M; b++) {
#pragma unroll
      for (int j = 0; j < H; j++) {
        const int i = b * 2 * H + j;
        bfly_gs(v[i], v[i + H], kTwE.p1i[M + b]);
      }
    }
  }
}

// Cyclic 32-point DFT with w = 2^6, decimation in frequency (natural in, bit-reversed out).
__device__ __forceinline__ void dft32_forward(u64 (&v)[32]) {
#pragma unroll
  for (int s = 0; s < 5; s++) {
    const int H = 16 >> s;
#pragma unroll
    for (int blk = 0; blk < 32; blk += 2 * H) {
#pragma unroll
      for (int j = 0; j < H; j++) bfly_gs(v[blk + j], v[blk + j + H], kTwE.dft[(j << s) & 31]);
    }
  }
}

// Inverse of dft32_forward (decimation in time; bit-reversed in, natural out; unscaled).
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

// Lane l, register k (residue brv5(k), coefficient l) -> lane u = brv5(k), register l.
__device__ __forceinline__ void transpose_forward(u64 (&v)[32], u64* reg, int l) {
#pragma unroll
  for (int k = 0; k < 32; k++) reg[brv5(k) * TROW + l] = v[k];
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < 32; j++) v[j] = reg[l * TROW + j];
  wave_lds_sync();
}

// Inverse of transpose_forward.
__device__ __forceinline__ void transpose_inverse(u64 (&v)[32], u64* reg, int l) {
#pragma unroll
  for (int j = 0; j < 32; j++) reg[j * TROW + l] = v[j];
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < 32; k++) v[k] = reg[l * TROW + brv5(k)];
  wave_lds_sync();
}

// Forward transform of this half's polynomial (values already residues mod p).
// tf is the [j][u] table psi_u^j (in LDS or global memory).
__device__ __forceinline__ void ntt_forward(u64 (&v)[32], const u64* tf, u64* reg, int l) {
  pass1_forward(v);
  transpose_forward(v, reg, l);
#pragma unroll
  for (int j = 1; j < 32; j++) v[j] = gl_mul(v[j], tf[j * 32 + l]);
  dft32_forward(v);
}

// Inverse transform (unscaled: returns N times the polynomial); ti is psi_u^-j.
__device__ __forceinline__ void ntt_inverse(u64 (&v)[32], const u64* ti, u64* reg, int l) {
  dft32_inverse(v);
#pragma unroll
  for (int j = 1; j < 32; j++) v[j] = gl_mul(v[j], ti[j * 32 + l]);
  transpose_inverse(v, reg, l);
  pass1_inverse(v);
}

// Gadget digit of a torus value at bit offset sh = 32 - 6r (r = 1..3): signed in [-32, 31],
// returned as a residue mod p. The rounding offset makes the l digits a round-to-nearest
// decomposition.
__device__ __forceinline__ u64 gadget_digit(u32 x, int sh) {
  const u32 t = x + DECOMP_OFFSET;
  const int32_t d = (int32_t)((t >> sh) & 63u) - 32;
  return gl_from_i32(d);
}

// Wave-cooperative external product: this half's polynomial of C (ext) D, added to acc.
// D holds this half's polynomial of the TRLWE operand (lanes 0-31: a, lanes 32-63: b);
// Cn is the TRGSW in the key layout above (already scaled by 1/N). Round k transforms
// digit k+1 of both halves (rows k and k+3 of C); each lane multiplies its transformed
// digits by the key entries of both output polynomials, keeps its own and passes the other
// to the partner lane 32 away. Key entries stream from memory in chunks of KCH slots, the
// next chunk in flight while the current one is used.
constexpr int KCH = 4;

__device__ __forceinline__ void external_product_acc(const u32 (&D)[32], const u64* __restrict__ Cn,
                                                     const u64* tf, const u64* ti, u64* reg, int lane,
                                                     u32 (&acc)[32]) {
  const int l = lane & 31;
  u64 x[32], sum[32];
#pragma unroll
  for (int s = 0; s < 32; s++) sum[s] = 0;
#pragma unroll 1
  for (int k = 0; k < GADGET_L; k++) {
    const u64* key = Cn + (size_t)k * (2 * 32 * 64) + lane;
    u64 ka[KCH], kb[KCH];
#pragma unroll
    for (int q = 0; q < KCH; q++) {
      ka[q] = __builtin_nontemporal_load(key + q * 64);
      kb[q] = __builtin_nontemporal_load(key + (32 + q) * 64);
    }
    const int sh = 32 - BG_BIT * (k + 1);
#pragma unroll
    for (int t = 0; t < 32; t++) x[t] = gadget_digit(D[t], sh);
    ntt_forward(x, tf, reg, l);
#pragma unroll
    for (int c = 0; c < 32 / KCH; c++) {
      u64 na[KCH], nb[KCH];
      if (c + 1 < 32 / KCH) {
#pragma unroll
        for (int q = 0; q < KCH; q++) {
          na[q] = __builtin_nontemporal_load(key + (KCH * (c + 1) + q) * 64);
          nb[q] = __builtin_nontemporal_load(key + (32 + KCH * (c + 1) + q) * 64);
        }
      }
#pragma unroll
      for (int q = 0; q < KCH; q++) {
        const int s = KCH * c + q;
        const u64 keep = gl_mul(x[s], ka[q]);
        const u64 send = gl_mul(x[s], kb[q]);
        const u64 recv = __shfl_xor(send, 32);
        sum[s] = gl_add(sum[s], gl_add(keep, recv));
      }
      __builtin_amdgcn_sched_barrier(0);
      if (c + 1 < 32 / KCH) {
#pragma unroll
        for (int q = 0; q < KCH; q++) {
          ka[q] = na[q];
          kb[q] = nb[q];
        }
      }
    }
  }
  ntt_inverse(sum, ti, reg, l);
#pragma unroll
  for (int t = 0; t < 32; t++) acc[t] += gl_lift_u32(gl_canon(sum[t]));
}

// Coefficient j of X^k * (mu, mu, ..., mu), k in [0, 2N).
__device__ __forceinline__ u32 rotated_testvector(int j, int k) {
  const bool wrap = j < (k & (RING_N - 1));
  const bool neg = wrap != (k >= RING_N);
  return neg ? (0u - MU) : MU;
}

// D = X^k * P - P for this half's polynomial (k in [0, 2N)), through the LDS region.
__device__ __forceinline__ void rotate_minus(const u32 (&P)[32], int k, u64* reg, int l, u32 (&D)[32]) {
  u32* buf = reinterpret_cast<u32*>(reg);
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
