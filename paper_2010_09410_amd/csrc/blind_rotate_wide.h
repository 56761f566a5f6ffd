// Latency form of the blind rotation: one gate per workgroup of three waves, wave k computing
// round k of every external product (gadget digit k+1 of both halves of X^a ACC - ACC, its
// forward transform and its key products). The three partial sums meet in LDS, and wave 0
// runs the inverse transform and the accumulator update. A step's critical path is one
// forward transform, one inverse transform and the exchange, instead of three forward
// transforms and one inverse, at the price of idle waves 1 and 2 during the inverse.
// Results are bit-identical to the one-wave form (exact integer arithmetic).
#pragma once
#include "vsp_internal.h"

namespace vsp {

constexpr int BRW_WAVES = GADGET_L;  // one wave per gadget level
// LDS per gate: the accumulator (2N u32) and one transpose region per wave; the regions of
// waves 1 and 2 are adjacent and double as the partial-sum exchange (32 slots x 64 lanes u64).
constexpr int BRW_GATE_U32 = 2 * RING_N + BRW_WAVES * WAVE_T_U32;
static_assert(2 * WAVE_T_U32 * 4 >= 32 * 64 * 8, "the exchange fits in two transpose regions");
static_assert(((2 * RING_N + WAVE_T_U32) * 4) % 8 == 0, "the exchange is 8-byte aligned");

constexpr size_t brw_lds_bytes() { return 2048 * 8 + (size_t)BRW_GATE_U32 * 4; }

// One round of an external product for this wave's digit level k: sum[s] receives, for this
// lane's output polynomial, the two key products of slot s (rows k and k + 3) reduced once.
template <class DigitSource>
__device__ __forceinline__ void external_round(DigitSource digits, int k, const u64* __restrict__ Cn, const u64* tf,
                                               u32* reg, int lane, u64 (&sum)[32]) {
  const int l = lane & 31;
  u64 x[32];
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
      sum[s] = gl_dot2(xa, kc[q].x, xb, kc[q].y);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (c + 1 < 32 / KCH) {
#pragma unroll
      for (int q = 0; q < KCH; q++) kc[q] = kn[q];
    }
  }
}

__global__ __launch_bounds__(BRW_WAVES * 64) void k_blind_rotate_wide(const u64* __restrict__ bkn,
                                                                      const u64* __restrict__ tw,
                                                                      const uint8_t* __restrict__ ops,
                                                                      const u32* __restrict__ abar,
                                                                      u32* __restrict__ tlwe1, u32* __restrict__ trlwe,
                                                                      uint64_t B, const u64* const* __restrict__ keytab,
                                                                      const uint16_t* __restrict__ kid) {
  extern __shared__ u64 lds[];
  u64* tws = lds;
  for (int i = threadIdx.x; i < 2048; i += BRW_WAVES * 64) tws[i] = tw[i];
  const uint64_t g = blockIdx.x;  // the grid has exactly B workgroups
  if (ops && !op_bootstraps(ops[g])) return;  // uniform over the workgroup: no barrier is skipped by half
  if (keytab) bkn = keytab[kid[g]];           // per-gate key (same value in every wave)
  const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // this wave's digit level
  const int lane = threadIdx.x & 63, l = lane & 31, h = lane >> 5;
  u32* gbase = reinterpret_cast<u32*>(lds + 2048);
  u64* xch = reinterpret_cast<u64*>(gbase + 2 * RING_N + WAVE_T_U32);
  const u32* ab = abar + g * TLWE0;
  if (k == 0) {
    const int bbar = (int)ab[LWE_N];
    const int k0 = (2 * RING_N - bbar) & (2 * RING_N - 1);
    u32* accs = gbase + h * RING_N;
#pragma unroll
    for (int t = 0; t < 32; t++) accs[l + 32 * t] = h ? rotated_testvector(l + 32 * t, k0) : 0u;
  }
  __syncthreads();
  for (int i = 0; i < LWE_N; i++) {
    const int a = (int)__builtin_amdgcn_readfirstlane(ab[i]);
    if (a == 0) continue;  // same value in every wave of the workgroup
    const int ln = opaque_lane(lane);
    const int li = ln & 31, hi = ln >> 5;
    u32* accs = gbase + hi * RING_N;
    u32* treg = gbase + 2 * RING_N + k * WAVE_T_U32 + hi * TREGION;
    auto digits = [&](int sh, u64 (&x)[32]) {
#pragma unroll
      for (int t = 0; t < 32; t++) {
        const int idx = (li + 32 * t - a) & (2 * RING_N - 1);
        u32 r = accs[idx & (RING_N - 1)];
        if (idx & RING_N) r = 0u - r;
        x[t] = gadget_digit(r - accs[li + 32 * t], sh);
      }
    };
    u64 sum[32];
    external_round(digits, k, bkn + (size_t)i * TRGSW_NTT_U64, tws, treg, ln, sum);
    __syncthreads();  // every wave is done with its transpose region and with ACC
    if (k == 2) {
#pragma unroll
      for (int s = 0; s < 32; s++) xch[s * 64 + ln] = sum[s];
    }
    __syncthreads();
    if (k == 1) {
#pragma unroll
      for (int s = 0; s < 32; s++) xch[s * 64 + ln] = gl_add(sum[s], xch[s * 64 + ln]);
    }
    __syncthreads();
    if (k == 0) {
#pragma unroll
      for (int s = 0; s < 32; s++) sum[s] = gl_add(sum[s], xch[s * 64 + ln]);
      u32 z[32];
      ntt_inverse_lift(sum, tws + 1024, treg, li, z);
#pragma unroll
      for (int t = 0; t < 32; t++)
        __hip_atomic_fetch_add(&accs[li + 32 * t], z[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    __syncthreads();  // the updated ACC is visible to the next step's digits
  }
  if (k != 0) return;
  const u32* accs = gbase + h * RING_N;
  if (trlwe) {
    u32* o = trlwe + g * 2 * RING_N + h * RING_N;
#pragma unroll
    for (int t = 0; t < 32; t++) o[l + 32 * t] = accs[l + 32 * t];
  }
  if (tlwe1) {
    // SampleExtract at 0: a'_0 = A_0, a'_j = -A_{N-j}; b' = B_0.
    u32* o = tlwe1 + g * TLWE1;
    if (h == 0) {
#pragma unroll
      for (int t = 0; t < 32; t++) {
        const int j = l + 32 * t;
        const u32 v = accs[j];
        o[(RING_N - j) & (RING_N - 1)] = (j == 0) ? v : 0u - v;
      }
    } else if (l == 0) {
      o[RING_N] = accs[0];
    }
  }
}

}  // namespace vsp
