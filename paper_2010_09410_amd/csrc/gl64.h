// Arithmetic modulo the NTT prime p = 2^64 - 2^32 + 1 on a 32-bit vector ALU.
//
// The ciphertext torus is Z/2^32; products of polynomials in Z[X]/(X^N+1) are computed
// exactly over Z by a negacyclic NTT modulo p and then reduced mod 2^32. This is exact
// because every coefficient of a gadget-digit (|d| <= 32) times torus (< 2^32) product,
// summed over 2l = 6 rows of N = 1024 terms, has absolute value below 6*1024*32*2^32 =
// 2^49.6 < p/2 (the paper's GPU library uses the same prime for its polynomial
// products, Sec. 6.2(a)).
//
// Values are kept "lazy": any 64-bit representative of the residue class (in [0, 2^64)),
// canonicalised to [0, p) only where an exact integer is needed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vsp {

typedef uint32_t u32;
typedef uint64_t u64;

constexpr u64 GL_P = 0xFFFFFFFF00000001ull;
constexpr u64 GL_EPS = 0xFFFFFFFFull;  // 2^64 mod p

// ---------------------------------------------------------------- compile-time helpers
constexpr u64 gl_mulmod_const(u64 a, u64 b) { return (u64)(((unsigned __int128)a * b) % GL_P); }
constexpr u64 gl_powmod_const(u64 b, u64 e) {
  u64 r = 1;
  b %= GL_P;
  while (e) {
    if (e & 1) r = gl_mulmod_const(r, b);
    b = gl_mulmod_const(b, b);
    e >>= 1;
  }
  return r;
}
// 2^e mod p for e in [0, 192): 2 has multiplicative order 192 (2^96 = -1).
constexpr u64 gl_pow2_const(int e) { return gl_powmod_const(2, (u64)(((e % 192) + 192) % 192)); }

// ---------------------------------------------------------------- device arithmetic
// a + b mod p for lazy a, b. A carry out of 2^64 is worth 2^64 = 2^32 - 1 (mod p); a second
// carry can only follow when both inputs were at or above p.
__device__ __forceinline__ u64 gl_add(u64 a, u64 b) {
  const u64 s = a + b;
  const u64 c1 = (s < a) ? GL_EPS : 0;
  const u64 s2 = s + c1;
  const u64 c2 = (s2 < c1) ? GL_EPS : 0;
  return s2 + c2;
}

// a - b mod p for lazy a, b (a borrow is worth -(2^32 - 1)).
__device__ __forceinline__ u64 gl_sub(u64 a, u64 b) {
  const u64 d = a - b;
  const u64 c1 = (a < b) ? GL_EPS : 0;
  const u64 d2 = d - c1;
  const u64 c2 = (d < c1) ? GL_EPS : 0;
  return d2 - c2;
}

// (hi:lo) mod p using 2^64 = 2^32 - 1 and 2^96 = -1: lo - hi_hi + hi_lo (2^32 - 1).
__device__ __forceinline__ u64 gl_reduce128(u64 lo, u64 hi) {
  const u32 hh = (u32)(hi >> 32), hl = (u32)hi;
  u64 t0 = lo - hh;
  if (lo < hh) t0 -= GL_EPS;  // cannot borrow twice: lo - hh + 2^64 > 2^32
  const u64 t1 = ((u64)hl << 32) - hl;
  u64 r = t0 + t1;
  if (r < t1) r += GL_EPS;    // cannot carry twice: t1 <= (2^32-1)^2
  return r;
}

// 64 x 64 -> 128-bit product from four 32 x 32 -> 64 multiply-adds.
__device__ __forceinline__ void mul128(u64 a, u64 b, u64& lo, u64& hi) {
  const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
  const u64 p00 = (u64)a0 * b0;
  const u64 t = (u64)a0 * b1 + (p00 >> 32);
  const u64 u = (u64)a1 * b0 + (u32)t;
  hi = (u64)a1 * b1 + (t >> 32) + (u >> 32);
  lo = (u << 32) | (u32)p00;
}

__device__ __forceinline__ u64 gl_mul(u64 a, u64 b) {
  u64 lo, hi;
  mul128(a, b, lo, hi);
  return gl_reduce128(lo, hi);
}

// x * 2^E mod p for a compile-time E in [0, 96), without a general multiply.
// Write x 2^E as 32-bit words w0..w4 of a 160-bit integer; then 2^64 = 2^32 - 1,
// 2^96 = -1 and 2^128 = -2^32 (mod p) fold it back to 64 bits.
__device__ __forceinline__ u64 gl_mul_pow2(u64 x, int E) {
  if (E == 0) return x;
  if (E <= 32) {
    // (hi:lo) = x << E with hi < 2^32: value = lo + hi (2^32 - 1).
    const u64 lo = (E == 32) ? (x << 32) : (x << E);
    const u64 hi = x >> (64 - E);
    const u64 t1 = (hi << 32) - hi;
    u64 r = lo + t1;
    if (r < t1) r += GL_EPS;
    return r;
  }
  if (E < 64) return gl_reduce128(x << E, x >> (64 - E));
  // E in [64, 96): F = E - 64, (w4:w3:w2) = x << F; value = w2 (2^32 - 1) - w3 - w4 2^32.
  const int F = E - 64;
  const u32 x0 = (u32)x, x1 = (u32)(x >> 32);
  const u32 w2 = (F == 0) ? x0 : (x0 << F);
  const u32 w3 = (F == 0) ? x1 : ((x1 << F) | (x0 >> (32 - F)));
  const u32 w4 = (F == 0) ? 0u : (x1 >> (32 - F));
  const u64 A = (u64)w2 << 32;
  const u64 B = ((u64)w4 << 32) + (u64)w2 + (u64)w3;  // < 2^63 + 2^33 < p
  const u64 d = A - B;
  return (A < B) ? d - GL_EPS : d;                    // one borrow at most (B < p)
}

// Canonical representative in [0, p).
__device__ __forceinline__ u64 gl_canon(u64 x) { return (x >= GL_P) ? x - GL_P : x; }

// A signed 32-bit integer as a residue mod p.
__device__ __forceinline__ u64 gl_from_i32(int32_t d) {
  return (d >= 0) ? (u64)d : (u64)((int64_t)d) - GL_EPS;  // 2^64 + d - (2^32 - 1) = p + d
}

// Exact lift of a canonical residue c to the integer z in (-p/2, p/2), reduced mod 2^32.
// As p = 1 (mod 2^32), c - p = c - 1 (mod 2^32).
__device__ __forceinline__ u32 gl_lift_u32(u64 c) {
  return (u32)c - (c > (GL_P >> 1) ? 1u : 0u);
}

}  // namespace vsp
