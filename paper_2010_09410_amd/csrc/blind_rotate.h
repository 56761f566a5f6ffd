// Blind-rotation kernel (device code only; its launcher lives with the other launchers).
// Kept in a file of its own so that its source fingerprint names exactly the code a
// profile of it measured.
#pragma once
#include "vsp_internal.h"

namespace vsp {

// One wave per gate. The accumulator lives in LDS (its a polynomial for lanes 0-31, b for
// lanes 32-63; coefficient l + 32 t belongs to lane l). ACC starts as (0, X^{-bbar} tv) with
// tv = mu everywhere; step i adds BK_i (ext) (X^{abar_i} ACC - ACC) (a CMUX between ACC and
// its rotation selected by the key bit s0_i); a step with abar_i = 0 has a zero difference,
// hence a zero product, and is skipped. LDS per workgroup: the twiddle tables, then per wave
// the accumulator (2 x 1024 u32) and the two transpose regions.
constexpr int BR_WAVE_U32 = 2 * RING_N + WAVE_T_U32;

constexpr size_t br_lds_bytes(int waves) { return 2048 * 8 + (size_t)waves * BR_WAVE_U32 * 4; }

// With keytab non-NULL gate g uses the bootstrapping key keytab[kid[g]] (clients with their
// own keys in one launch), else bkn.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_blind_rotate(const u64* __restrict__ bkn, const u64* __restrict__ tw,
                                                             const uint8_t* __restrict__ ops,
                                                             const u32* __restrict__ abar, u32* __restrict__ tlwe1,
                                                             u32* __restrict__ trlwe, uint64_t B,
                                                             const u64* const* __restrict__ keytab,
                                                             const uint16_t* __restrict__ kid) {
  extern __shared__ u64 lds[];
  u64* tws = lds;
  for (int i = threadIdx.x; i < 2048; i += WAVES * 64) tws[i] = tw[i];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t g = (uint64_t)blockIdx.x * WAVES + wave;
  if (g >= B) return;
  if (ops && !op_bootstraps(ops[g])) return;
  if (keytab) bkn = keytab[__builtin_amdgcn_readfirstlane(kid[g])];
  const int lane = threadIdx.x & 63, l = lane & 31, h = lane >> 5;
  u32* wbase = reinterpret_cast<u32*>(lds + 2048) + wave * BR_WAVE_U32;
  const u32* ab = abar + g * TLWE0;
  const int bbar = (int)ab[LWE_N];
  const int k0 = (2 * RING_N - bbar) & (2 * RING_N - 1);
  {
    u32* accs = wbase + h * RING_N;
#pragma unroll
    for (int t = 0; t < 32; t++) accs[l + 32 * t] = h ? rotated_testvector(l + 32 * t, k0) : 0u;
  }
  wave_lds_sync();
  for (int i = 0; i < LWE_N; i++) {
    const int a = (int)__builtin_amdgcn_readfirstlane(ab[i]);
    if (a == 0) continue;
    const int ln = opaque_lane(lane);
    const int li = ln & 31, hi = ln >> 5;
    u32* accs = wbase + hi * RING_N;
    u32* treg = wbase + 2 * RING_N + hi * TREGION;
    // digits of X^a ACC - ACC, recomputed from the LDS accumulator in every round
    auto digits = [&](int sh, u64 (&x)[32]) {
#pragma unroll
      for (int t = 0; t < 32; t++) {
        const int idx = (li + 32 * t - a) & (2 * RING_N - 1);
        u32 r = accs[idx & (RING_N - 1)];
        if (idx & RING_N) r = 0u - r;
        x[t] = gadget_digit(r - accs[li + 32 * t], sh);
      }
    };
    u32 z[32];
    external_product(digits, bkn + (size_t)i * TRGSW_NTT_U64, tws, tws + 1024, treg, ln, z);
#pragma unroll
    for (int t = 0; t < 32; t++)
      __hip_atomic_fetch_add(&accs[li + 32 * t], z[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    wave_lds_sync();
  }
  const u32* accs = wbase + h * RING_N;
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
