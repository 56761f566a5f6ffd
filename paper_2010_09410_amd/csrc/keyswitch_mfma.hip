// Identity key switch on the matrix cores (Sec. 2.1.2, Sample Extraction and Identity Key
// Switching): out = (0, b') - sum_{j < N, p < t} KSK[j][p][v_{j,p}], v_{j,p} the p-th base-4
// digit of a'_j rounded to 16 bits, written as a matrix product over the batch. For a gate g,
// row (j, p, v) of its one-hot operand is 1 where v = v_{g,j,p}; the key rows (the v = 0 row is
// zero) are the other operand, split into four balanced signed bytes and folded by Horner's
// rule in the accumulators exactly as in the matrix-core blind rotation (int32 wrap-around is
// arithmetic mod 2^32; per byte plane a sum has at most 8192 nonzero terms of magnitude at
// most 128).
//
// The 32 rows (p, v) of one j form one 32-deep block of the product: lane (m, kh) of the
// operand of gate m holds p = 4 kh .. 4 kh + 3 as four words 1 << (8 v_{g,j,p}), built from
// a'_j in registers. The key bytes are stored in the lane order of the other operand,
// [plane][j][column tile][lane][16], so a wave's load of one block is 1 KiB contiguous.
// A workgroup of four waves takes 128 gates and 64 output columns; wave s takes j in
// [256 s, 256 s + 256), and the four partial sums meet in LDS. The digits of a gate depend only
// on the top 16 bits of a'_j + 2^15. Rows past the batch get digits of 0 (the zero key row);
// a gate that does not bootstrap is computed like the others and its output is not written.
#include "vsp_internal.h"

namespace vsp {

typedef int ks_v4i __attribute__((ext_vector_type(4)));
typedef int ks_v16i __attribute__((ext_vector_type(16)));

constexpr int KM_CT = (TLWE0 + 31) / 32;           // 20 column tiles of 32 (631 columns)
constexpr int KM_PLANES = 4;
constexpr size_t KM_KEY_BYTES = (size_t)KM_PLANES * RING_N * KM_CT * 64 * 16;
constexpr int KM_GATES = 128;                      // gates per workgroup (four tiles of 32)
constexpr int KM_COLS = 2;                         // column tiles per workgroup
constexpr int KM_SPLIT = 4;                        // waves per workgroup, one j range each
constexpr int KM_JR = RING_N / KM_SPLIT;

// KB[b][j][ct][lane][16]: lane (n, kh), byte 4 w + v holds byte b of KSK[j][4 kh + w][v][32 ct + n]
// (zero for v = 0 and past column n).
__global__ __launch_bounds__(256) void k_ks_mfkey(const u32* __restrict__ ksk, int8_t* __restrict__ KB) {
  const uint64_t id = (uint64_t)blockIdx.x * 256 + threadIdx.x;  // one word (four bytes) each
  if (id >= KM_KEY_BYTES / 4) return;
  const int w = (int)(id & 3), lane = (int)((id >> 2) & 63);
  const uint64_t rest = id >> 8;
  const int ct = (int)(rest % KM_CT);
  const uint64_t bj = rest / KM_CT;
  const int j = (int)(bj % RING_N), b = (int)(bj / RING_N);
  const int n = lane & 31, kh = lane >> 5, c = 32 * ct + n, p = 4 * kh + w;
  u32 word = 0;
#pragma unroll
  for (int v = 0; v < 4; v++) {
    u32 x = (c < TLWE0) ? ksk[(((size_t)j * KS_T + p) * 4 + v) * TLWE0 + c] : 0u;
    int8_t cb = 0;
    for (int bb = 0; bb <= b; bb++) {
      cb = (int8_t)(x & 255u);  // x = cb (mod 256), cb in [-128, 127]
      x = (x - (u32)(int32_t)cb) >> 8;
    }
    word |= ((u32)(uint8_t)cb) << (8 * v);
  }
  reinterpret_cast<u32*>(KB)[id] = word;
}

// The top 16 bits of each rounded a'_j (all the digits need) are staged per wave in LDS as
// [j][gate] u16 for chunks of KM_JC coefficients, rows padded to spread the banks, with 32
// gates' loads in flight at once; the key operands stream from global memory three blocks
// ahead. Every load is unconditional (gate index clamped, the last three key blocks re-read
// and unused): a guarded load becomes a branch, after which the compiler waits for it.
constexpr int KM_JC = 64;
constexpr int KM_HROW = KM_GATES + 2;  // u16 per staged row

__global__ __launch_bounds__(256, 2) void k_ks_mfma(const int8_t* __restrict__ KB, const uint8_t* __restrict__ ops,
                                                     const u32* __restrict__ tlwe1, const u32* __restrict__ idxo,
                                                     u32* __restrict__ out, uint64_t B) {
  __shared__ uint16_t hs[KM_SPLIT][KM_JC][KM_HROW];
  static_assert(sizeof(hs) >= (size_t)4 * KM_COLS * 16 * 64 * 4, "the partial sums fit in the staging area");
  const int s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int m = lane & 31, kh = lane >> 5;
  const uint64_t g0 = (uint64_t)blockIdx.x * KM_GATES;
  const int ct0 = blockIdx.y * KM_COLS;
  const int j0 = s * KM_JR;
  const uint4* kb = reinterpret_cast<const uint4*>(KB) + lane;  // + ((b * N + j) * KM_CT + ct) * 64
  ks_v16i acc[4][KM_COLS];
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int u = 0; u < KM_COLS; u++)
#pragma unroll
      for (int x = 0; x < 16; x++) acc[t][u][x] = 0;
  uint16_t(*h)[KM_HROW] = hs[s];
  for (int b = KM_PLANES - 1; b >= 0; b--) {
    const uint4* kp = kb + ((size_t)b * RING_N * KM_CT + ct0) * 64;
    auto ldb = [&](int j, uint4 (&r)[KM_COLS]) {
#pragma unroll
      for (int u = 0; u < KM_COLS; u++) r[u] = kp[((size_t)j * KM_CT + u) * 64];
    };
    uint4 bq[4][KM_COLS];  // block j in slot (j - j0) mod 4
    ldb(j0, bq[0]);
    ldb(j0 + 1, bq[1]);
    ldb(j0 + 2, bq[2]);
    for (int jc = j0; jc < j0 + KM_JR; jc += KM_JC) {
      // stage the digits' source bits of this wave's gates for jc .. jc + KM_JC - 1
      wave_lds_sync();
#pragma unroll 1
      for (int q0 = 0; q0 < KM_GATES; q0 += 32) {
        u32 v[32];
#pragma unroll
        for (int q = 0; q < 32; q++) {
          const uint64_t g = g0 + q0 + q;
          v[q] = tlwe1[(g < B ? g : 0) * TLWE1 + jc + lane];
        }
#pragma unroll
        for (int q = 0; q < 32; q++)
          h[lane][q0 + q] = (g0 + q0 + q < B) ? (uint16_t)((v[q] + (1u << 15)) >> 16) : (uint16_t)0;
      }
      wave_lds_sync();
      for (int jj = 0; jj < KM_JC; jj += 4) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int j = jc + jj + r;
          ldb(j + 3 < j0 + KM_JR ? j + 3 : j0 + KM_JR - 1, bq[(r + 3) & 3]);
          ks_v4i bv[KM_COLS];
#pragma unroll
          for (int u = 0; u < KM_COLS; u++)
            bv[u] = ks_v4i{(int)bq[r][u].x, (int)bq[r][u].y, (int)bq[r][u].z, (int)bq[r][u].w};
#pragma unroll
          for (int t = 0; t < 4; t++) {
            const u32 hv = h[jj + r][32 * t + m];
            ks_v4i av;
#pragma unroll
            for (int w = 0; w < 4; w++) av[w] = (int)(1u << (8 * ((hv >> (14 - 2 * (4 * kh + w))) & 3u)));
#pragma unroll
            for (int u = 0; u < KM_COLS; u++)
              acc[t][u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv[u], acc[t][u], 0, 0, 0);
          }
        }
      }
    }
    if (b > 0) {
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int u = 0; u < KM_COLS; u++)
#pragma unroll
          for (int x = 0; x < 16; x++) acc[t][u][x] = (int)((u32)acc[t][u][x] << 8);
    }
  }
  // the partial sums of waves 1..3 through LDS to wave 0, one wave at a time
  int(*red)[64] = reinterpret_cast<int(*)[64]>(&hs[0][0][0]);
  __syncthreads();  // every wave is done with its staging rows
  for (int q = 1; q < KM_SPLIT; q++) {
    if (s == q) {
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int u = 0; u < KM_COLS; u++)
#pragma unroll
          for (int x = 0; x < 16; x++) red[(t * KM_COLS + u) * 16 + x][lane] = acc[t][u][x];
    }
    __syncthreads();
    if (s == 0) {
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int u = 0; u < KM_COLS; u++)
#pragma unroll
          for (int x = 0; x < 16; x++) acc[t][u][x] += red[(t * KM_COLS + u) * 16 + x][lane];
    }
    __syncthreads();
  }
  if (s != 0) return;
  // result (gate, column): lane n + 32 kh, register x: gate row 8 (x / 4) + 4 kh + x % 4 of the
  // tile, column 32 ct + n. Per tile, the gate types, output rows and b' of the lane's 16 gates
  // are loaded together first (unconditionally, gate index clamped).
  const bool has_b = ct0 + KM_COLS > LWE_N / 32;  // this workgroup writes column n (the b part)
#pragma unroll
  for (int t = 0; t < 4; t++) {
    uint8_t opv[16];
    u32 rov[16], bv[16];
#pragma unroll
    for (int x = 0; x < 16; x++) {
      const uint64_t g = g0 + 32 * t + 8 * (x >> 2) + 4 * kh + (x & 3);
      opv[x] = 0;  // a bootstrapping gate type
      rov[x] = (u32)g;
      bv[x] = 0;
    }
    if (ops) {
#pragma unroll
      for (int x = 0; x < 16; x++) {
        const uint64_t g = g0 + 32 * t + 8 * (x >> 2) + 4 * kh + (x & 3);
        opv[x] = ops[g < B ? g : 0];
      }
    }
    if (idxo) {
#pragma unroll
      for (int x = 0; x < 16; x++) {
        const uint64_t g = g0 + 32 * t + 8 * (x >> 2) + 4 * kh + (x & 3);
        rov[x] = idxo[g < B ? g : 0];
      }
    }
    if (has_b) {
#pragma unroll
      for (int x = 0; x < 16; x++) {
        const uint64_t g = g0 + 32 * t + 8 * (x >> 2) + 4 * kh + (x & 3);
        bv[x] = tlwe1[(g < B ? g : 0) * TLWE1 + RING_N];
      }
    }
#pragma unroll
    for (int x = 0; x < 16; x++) {
      const uint64_t g = g0 + 32 * t + 8 * (x >> 2) + 4 * kh + (x & 3);
      if (g >= B || !op_bootstraps(opv[x])) continue;
#pragma unroll
      for (int u = 0; u < KM_COLS; u++) {
        const int c = 32 * (ct0 + u) + m;
        if (c >= TLWE0) continue;
        out[(uint64_t)rov[x] * TLWE0 + c] = ((c == LWE_N) ? bv[x] : 0u) - (u32)acc[t][u][x];
      }
    }
  }
}

size_t ks_mf_key_bytes() { return KM_KEY_BYTES; }

hipError_t launch_ks_mfkey(const uint32_t* ksk, int8_t* KB, hipStream_t st) {
  hipLaunchKernelGGL(k_ks_mfkey, dim3((unsigned)(KM_KEY_BYTES / 4 / 256)), dim3(256), 0, st, ksk, KB);
  return hipGetLastError();
}

hipError_t launch_keyswitch_mfma(const int8_t* KB, const uint8_t* ops, const uint32_t* tlwe1, const uint32_t* idxo,
                                 uint32_t* out, uint64_t B, hipStream_t st) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ks_mfma, dim3((unsigned)((B + KM_GATES - 1) / KM_GATES), KM_CT / KM_COLS), dim3(256), 0, st, KB,
                     ops, tlwe1, idxo, out, B);
  return hipGetLastError();
}

}  // namespace vsp
