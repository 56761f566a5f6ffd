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

// a + t mod p for lazy a and t <= p: a carry can then happen only once, because the wrapped
// sum is below t.
__device__ __forceinline__ u64 gl_add_c(u64 a, u64 t) {
  const u64 s = a + t;
  return s + ((s < t) ? GL_EPS : 0);
}

// a - t mod p for lazy a and t <= p: after a borrow the difference is at least 2^64 - p.
__device__ __forceinline__ u64 gl_sub_c(u64 a, u64 t) {
  const u64 d = a - t;
  return d - ((a < t) ? GL_EPS : 0);
}

// Product modulo p (lazy result). The 128-bit product is (hi:lo); with hi = hh 2^32 + hl,
// 2^64 = 2^32 - 1 and 2^96 = -1 give lo + hl (2^32 - 1) - hh. hl (2^32 - 1) <= 2^64 - 2^33 + 1,
// so the sum carries at most once and the difference borrows at most once.
__device__ __forceinline__ u64 gl_mul(u64 a, u64 b) {
  const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
  const u64 p00 = (u64)a0 * b0;
  const u64 t = (u64)a0 * b1 + (p00 >> 32);
  const u64 u = (u64)a1 * b0 + (u32)t;
  const u64 hi = (u64)a1 * b1 + (t >> 32) + (u >> 32);
  const u64 lo = (u << 32) | (u32)p00;
  const u32 hh = (u32)(hi >> 32), hl = (u32)hi;
  const u64 tl = (u64)hl * GL_EPS;
  u64 r = lo + tl;
  r += (r < tl) ? GL_EPS : 0;
  const u64 r2 = r - hh;
  return r2 - ((r < hh) ? GL_EPS : 0);
}

// x0 k0 + x1 k1 mod p (lazy result) with one reduction: the two 128-bit products are added
// as a 129-bit integer (top:hi:lo); with hi = hh 2^32 + hl, 2^64 = 2^32 - 1, 2^96 = -1 and
// 2^128 = -2^32 it is lo + hl (2^32 - 1) - (hh + top 2^32), and the same single carry and
// single borrow fixes as in gl_mul apply (hh + top 2^32 < 2^33).
__device__ __forceinline__ u64 gl_dot2(u64 x0, u64 k0, u64 x1, u64 k1) {
  u64 l0, h0, l1, h1;
  {
    const u32 a0 = (u32)x0, a1 = (u32)(x0 >> 32), b0 = (u32)k0, b1 = (u32)(k0 >> 32);
    const u64 p00 = (u64)a0 * b0;
    const u64 t = (u64)a0 * b1 + (p00 >> 32);
    const u64 u = (u64)a1 * b0 + (u32)t;
    h0 = (u64)a1 * b1 + (t >> 32) + (u >> 32);
    l0 = (u << 32) | (u32)p00;
  }
  {
    const u32 a0 = (u32)x1, a1 = (u32)(x1 >> 32), b0 = (u32)k1, b1 = (u32)(k1 >> 32);
    const u64 p00 = (u64)a0 * b0;
    const u64 t = (u64)a0 * b1 + (p00 >> 32);
    const u64 u = (u64)a1 * b0 + (u32)t;
    h1 = (u64)a1 * b1 + (t >> 32) + (u >> 32);
    l1 = (u << 32) | (u32)p00;
  }
  const u64 lo = l0 + l1;
  const u64 hs = h0 + h1;
  const u64 hi = hs + (lo < l0 ? 1u : 0u);
  const bool top = (hs < h0) | (hi < hs);  // at most one of the two carries happens
  const u32 hh = (u32)(hi >> 32), hl = (u32)hi;
  const u64 tl = (u64)hl * GL_EPS;
  u64 r = lo + tl;
  r += (r < tl) ? GL_EPS : 0;
  const u64 sub = (u64)hh + (top ? (1ull << 32) : 0);
  const u64 r2 = r - sub;
  return r2 - ((r < sub) ? GL_EPS : 0);
}

// x * 2^E mod p for a compile-time E in [0, 96), returned canonical (in [0, p)). Write
// x 2^E as 32-bit words of a 160-bit integer and fold it back with 2^64 = 2^32 - 1 and
// 2^96 = -1:
//  E < 32:  x 2^E = L + w 2^64 (L the low 64 bits, w the top E bits) = L + w (2^32 - 1).
//           w (2^32 - 1) < 2^63, so after a carry the sum is below 2^63; without one it may
//           lie in [p, 2^64). Both cases are fixed by adding 2^32 - 1 once.
//  E >= 64: with F = E - 64 and (w4:w3:w2) = x 2^F, x 2^E = w2 (2^32 - 1) - (w4:w3), where
//           w2 (2^32 - 1) < p; one conditional subtraction of 2^32 - 1 after a borrow lands
//           in [0, p).
//  else:    with F = E - 32 and (w2:w1:w0) = x 2^F, x 2^E = [w0 2^32 + w1 (2^32 - 1)] - w2,
//           the bracket made canonical as in the first case, then w2 subtracted as in the
//           second.
__device__ __forceinline__ u64 gl_mul_pow2(u64 x, int E) {
  if (E == 0) return (x >= GL_P) ? x + GL_EPS : x;
  if (E < 32) {
    const u64 t = (u64)(u32)(x >> (64 - E)) * GL_EPS;
    const u64 r = (x << E) + t;
    return r + (((r < t) | (r >= GL_P)) ? GL_EPS : 0);
  }
  if (E >= 64) {
    const int F = E - 64;
    const u64 sh = x << F;
    const u32 w4 = F ? (u32)(x >> (64 - F)) : 0u;
    const u64 A = (u64)(u32)sh * GL_EPS;
    const u64 Bv = ((u64)w4 << 32) | (sh >> 32);
    const u64 r = A - Bv;
    return r - ((A < Bv) ? GL_EPS : 0);
  }
  const int F = E - 32;
  const u64 sh = x << F;
  const u32 w2 = F ? (u32)(x >> (64 - F)) : 0u;
  const u64 t = (u64)(u32)(sh >> 32) * GL_EPS;
  u64 a = (sh << 32) + t;
  a += ((a < t) | (a >= GL_P)) ? GL_EPS : 0;
  const u64 r = a - w2;
  return r - ((a < (u64)w2) ? GL_EPS : 0);
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
