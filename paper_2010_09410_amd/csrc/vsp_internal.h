// Internal declarations of libvsp: the context object, device kernels' launchers, errors.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/vsp.h"
#include "ntt.h"

namespace vsp {

// Row lengths of TLWE ciphertexts under the LWE key (n + 1) and the extracted ring key (N + 1).
constexpr int TLWE0 = LWE_N + 1;
constexpr int TLWE1 = RING_N + 1;

// Largest number of gates (bootstraps, key switches) in one launch sequence; larger calls are
// split so that every grid stays far below the 2^31 workgroup limit.
constexpr uint64_t kMaxLaunch = 1ull << 22;

// Internal opcode: bootstrap the first input unchanged (refresh of a noisy TLWE).
constexpr uint8_t OP_IDENT = 16;
// Internal opcode: a padding entry of a batch (no input read, no output written, no bootstrap).
constexpr uint8_t OP_SKIP = 17;

__host__ __device__ inline bool op_bootstraps(uint32_t op) { return op < 8 || op == OP_IDENT; }

// Device-side error flags (bits), read back by vsp_context_sync.
constexpr int DEVERR_BAD_OP = 1;

// Blind-rotation forms: 4 or 8 gates per workgroup at one wave per gate, 3 for one gate per
// workgroup on three waves (the latency form), 32 for the matrix-core form (int8 MFMA products
// over tiles of MF_TILE gates, one workgroup per tile and output polynomial, one launch per
// step), and 33 for its split form (the products of a step cut into workgroups per tile,
// output polynomial, sub-product and group of TRGSW rows, and for single rows also per range
// of byte planes, for batches too small to fill the chip; two launches per step).
constexpr int kBrShapes = 5;
constexpr int kBrWaveChoices[kBrShapes] = {4, 8, 3, 32, 33};
constexpr int MF_TILE = 32;
inline bool br_matrix_form(int waves) { return waves == 32 || waves == 33; }
// Workgroup counts per (tile, output, sub-product) of the split form: 1, 2, 3 or 6 groups of
// TRGSW rows, or one row per workgroup with the four byte planes in 2 (12) or 4 (24) ranges;
// the shares go into ACC with integer atomics. -1, -2, -3, -6, -12, -24: the same workgroups
// with the shares stored as partial sums and added up by the next digit launch (batches of at
// most kPartTiles tiles, kPartSmallTiles for -12 and -24; larger ones use the atomics).
constexpr int kSplitGroupChoices[12] = {1, 2, 3, 6, 12, 24, -1, -2, -3, -6, -12, -24};
constexpr int kPartTiles = 96;
constexpr int kPartSmallTiles = 8;
inline bool split_groups_valid(int g) {
  for (int c : kSplitGroupChoices)
    if (g == c) return true;
  return false;
}
// Row groups of the split form for B gates on a chip of `cus` compute units: the fewest that
// give about three workgroups of four waves per compute unit.
inline int mf_split_groups(uint64_t B, int cus) {
  const uint64_t units = (B + MF_TILE - 1) / MF_TILE * 2 * 3;  // tiles x outputs x sub-products
  for (int g : {1, 2, 3})
    if (units * (uint64_t)g >= 3ull * (uint64_t)(cus > 0 ? cus : 256)) return g;
  return 6;
}

// Batch-size buckets: bucket b holds batches with kBucket[b-1] < B <= kBucket[b]; the last
// one also holds every larger batch.
constexpr int kTuneBuckets = 7;
constexpr uint64_t kBucket[kTuneBuckets] = {1, 16, 64, 256, 1024, 2048, 4096};
// Batch sizes at which the split matrix-core form is timed (its time is interpolated between).
constexpr int kSplitPts = 13;
constexpr uint64_t kSplitAt[kSplitPts] = {1, 16, 64, 256, 512, 768, 1024, 1280, 1536, 1792, 2048, 3072, 4096};

// Launch choices, set by vsp_autotune or left at the defaults. Every choice gives
// bit-identical results.
//  * Blind rotation: a gate is one wave from start to end, so a batch of B gates takes
//    ceil(B / br_cap[s]) rounds of br_round_ms[s] with shape s, where br_cap[s] is the number
//    of gates the whole GPU holds at once (occupancy x compute units x gates per group) and
//    br_round_ms[s] the time of one full round. The split matrix-core form is timed instead
//    at the sizes kSplitAt (split_ms[k], with the fastest row-group count split_groups[k]) and
//    estimated in between by linear interpolation (beyond the last size: in proportion), with
//    a 3% margin above 1,280 gates.
//    The shape with the fewer milliseconds wins (ties: the 8-gate workgroup). br_force[b] != 0
//    pins the shape for bucket b.
//  * Key switch: per bucket, form 0 gathers key rows per gate, 1 reads them once per tile of
//    gates and selects in registers, 2 stages them through LDS for a tile of gates and splits
//    the j range over workgroups, 3 runs on the matrix cores (one-hot digit rows times the
//    key's byte planes).
struct Tuning {
  uint64_t br_cap[kBrShapes] = {1024, 2048, 512, 4096, MF_TILE};
  float br_round_ms[kBrShapes] = {1.0f, 1.482f, 0.75f, 2.33f, 0.337f};
  // split form, at the sizes kSplitAt: time in the same units as br_round_ms, and row groups
  // (0: the count that fills the chip, mf_split_groups). The defaults are relative times
  // measured on an MI355X (one 4-gate-workgroup round = 1).
  float split_ms[kSplitPts] = {0.114f, 0.190f, 0.246f, 0.355f, 0.505f, 0.670f, 0.857f, 0.916f, 1.253f, 1.333f, 1.399f,
                               2.180f, 2.530f};
  int split_groups[kSplitPts] = {24, 12, -6, -6, -2, -3, -2, -1, -2, -2, -2, -2, 1};
  int br_force[kTuneBuckets] = {0, 0, 0, 0, 0, 0, 0};
  int ks_form[kTuneBuckets] = {2, 2, 2, 2, 3, 3, 3};
  bool tuned = false;
  static int bucket(uint64_t B) {
    int b = 0;
    while (b + 1 < kTuneBuckets && B > kBucket[b]) b++;
    return b;
  }
  // with ntt_only, the best of the NTT forms (for launches that cannot take the matrix-core
  // forms: another key, or no workspace)
  int br_waves(uint64_t B, bool ntt_only = false) const {
    const int f = br_force[bucket(B)];
    if (f && !(ntt_only && br_matrix_form(f))) return f;
    int best = 1;
    double best_ms = 0;
    for (int s : {1, 0, 2, 3, 4}) {
      if (ntt_only && s >= 3) continue;
      const uint64_t cap = br_cap[s] ? br_cap[s] : 1;
      double ms = (double)((B + cap - 1) / cap) * br_round_ms[s];
      // above 1,280 gates the split form's time deviates from the interpolation by a few
      // percent between neighbouring sizes (measured: workgroup balance), so it must win by 3%
      if (s == 4) ms = split_estimate(B) * (B > kSplitAt[7] ? 1.03 : 1.0);
      if (s == 1 || ms < best_ms) {
        best = s;
        best_ms = ms;
      }
    }
    return kBrWaveChoices[best];
  }
  int ks_form_for(uint64_t B) const { return ks_form[bucket(B)]; }
  static int split_point(uint64_t B) {  // the first timed size at or above B (else the last)
    int k = 0;
    while (k + 1 < kSplitPts && B > kSplitAt[k]) k++;
    return k;
  }
  double split_estimate(uint64_t B) const {
    const int k = split_point(B);
    if (B >= kSplitAt[kSplitPts - 1]) return (double)split_ms[kSplitPts - 1] * (double)B / kSplitAt[k];
    if (k == 0) return split_ms[0];
    const double f = (double)(B - kSplitAt[k - 1]) / (double)(kSplitAt[k] - kSplitAt[k - 1]);
    return split_ms[k - 1] + f * (split_ms[k] - split_ms[k - 1]);
  }
  int split_groups_for(uint64_t B, int cus) const {
    const int g = split_groups[split_point(B)];
    return g ? g : mf_split_groups(B, cus);
  }
};

// Growable device scratch owned by a context.
struct Scratch {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Event pairs bracketing instrumented launches (kernel classes: blind rotation, key switch,
// prologue, and the step kernels of the matrix-core blind rotation, whose pair brackets the
// whole sequence of one blind rotation's step launches). Only eager calls from the caller's
// thread record them (not launches under stream capture, nor the server's worker thread).
constexpr int kProfClasses = 4;
struct ProfEvent {
  hipEvent_t e0, e1;
  uint32_t launches;  // kernel launches between e0 and e1
};
struct Profile {
  bool on = false;
  int period = 1;                  // instrument every period-th launch of each class
  uint64_t seen[kProfClasses] = {};  // launches of each class since enabling
  std::vector<ProfEvent> ev[kProfClasses];
};

}  // namespace vsp

// A client's key set converted for the device: bootstrapping key in the NTT domain and the
// key-switching key with zero rows (layouts as in vsp_context).
struct vsp_keyset {
  vsp_context* ctx = nullptr;
  uint64_t* bkn = nullptr;
  uint32_t* ksk = nullptr;
  int8_t* mf_key = nullptr;  // byte-plane forms for the matrix-core blind rotation and key switch
  int8_t* ks_mf = nullptr;
};

struct vsp_context {
  int device = 0;
  int cus = 1;                    // compute units of the device
  int8_t* mf_key = nullptr;       // bootstrapping key as balanced-byte Toeplitz rows (matrix-core form)
  int8_t* ks_mf = nullptr;        // key-switching key as balanced bytes in MFMA operand order (key-switch form 3)
  uint64_t* bkn = nullptr;        // bootstrapping key, NTT domain: [n][TRGSW_NTT_U64]
  uint32_t* ksk = nullptr;        // key-switching key [N][t][4][n+1]; digit value 0 points at a zero row
  uint64_t* tw = nullptr;         // psi_u^j [32][32] then psi_u^-j [32][32]
  int* dev_err = nullptr;         // device error flags
  vsp::Scratch abar, tlwe1, ntt_sel, mem_a, mem_b, mem_c, mem_d, mf_work;
  vsp::Tuning tune;
  mutable vsp::Profile prof;     // instrumentation, also recorded by launches on a const context
  std::mutex mu;                  // serialises scratch growth
};

namespace vsp {

// Thread-local error text and status helpers.
vsp_status fail(vsp_status s, const std::string& msg);
vsp_status hip_fail(hipError_t e, const char* what);
#define VSP_HIP(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return vsp::hip_fail(e_, #call); \
  } while (0)

// Returns VSP_OK if [p, p + bytes) lies inside one device allocation on ctx's device.
vsp_status check_device_range(const vsp_context* ctx, const void* p, size_t bytes, const char* name);
vsp_status check_no_overlap(const void* a, size_t abytes, const void* b, size_t bbytes, const char* what);

// Converts host keys (BK torus [n][2l][2][N], KSK [N][t][3][n+1]) into freshly allocated device
// buffers in the kernels' layouts; on failure nothing stays allocated.
vsp_status upload_keys(const vsp_context* ctx, const uint32_t* bk_host, const uint32_t* ksk_host, uint64_t** bkn,
                       uint32_t** ksk, int8_t** mf_key = nullptr, int8_t** ks_mf = nullptr);

// Grows a scratch buffer to at least `bytes` (synchronising the device before freeing).
vsp_status scratch_reserve(vsp_context* ctx, Scratch& s, size_t bytes);

// Records an event pair around `launches` launches of kernel class `which` when profiling is
// on and the stream is not being captured.
struct ProfScope {
  const vsp_context* ctx;
  int which;
  hipStream_t st;
  hipEvent_t e1 = nullptr;
  ProfScope(const vsp_context* c, int w, hipStream_t s, uint32_t launches = 1);
  ~ProfScope();
};

// ---------------------------------------------------------------- launchers (kernels.hip)
hipError_t init_kernel_attributes();
// Gates the device runs at once with each blind-rotation shape (resident groups x CUs x waves).
hipError_t blind_rotate_capacity(int device, uint64_t (&cap)[kBrShapes]);
// Torus TRGSW [count][2l][2][N] -> key layout [count][TRGSW_NTT_U64], scaled by 1/N.
hipError_t launch_trgsw_to_ntt(const vsp_context* ctx, const uint32_t* src, uint64_t* dst, uint64_t count,
                               hipStream_t st);
// Gate linear combination + modulus switch (abar [B][n+1]); NOT / invalid ops write out directly.
// idx0/idx1/idxo (optional) gather inputs and scatter outputs by wire id (stride n+1).
// With allow_not false, NOT is reported as an invalid opcode (TRLWE-output bootstrapping).
hipError_t launch_gate_prologue(const vsp_context* ctx, const uint8_t* ops, const uint32_t* in0, const uint32_t* in1,
                                const uint32_t* idx0, const uint32_t* idx1, const uint32_t* idxo, uint32_t* abar,
                                uint32_t* out, uint64_t B, hipStream_t st, bool allow_not = true);
// The same opcode for every gate, one input (e.g. OP_IDENT for a refresh bootstrap).
hipError_t launch_gate_prologue_uniform(const vsp_context* ctx, uint32_t op, const uint32_t* in0, uint32_t* abar,
                                        uint64_t B, hipStream_t st);
// Homomorphic MUX pieces: the 2B prologue rows (AND(s, c1), then ANDNOT(c0, s)) and the sum of
// the two extracted halves plus (0, mu) into the first B rows of t [2B][N+1].
hipError_t launch_mux_prologue(const uint32_t* sel, const uint32_t* in1, const uint32_t* in0, uint32_t* abar,
                               uint64_t B, hipStream_t st);
hipError_t launch_mux_combine(uint32_t* t, uint64_t B, hipStream_t st);
// Blind rotation of B gates (abar from the prologue). Writes SE_0 (TLWE1 [B][N+1]) and/or
// the accumulator (TRLWE [B][2][N]). waves: a shape of kBrWaveChoices, <= 0 the tuned choice.
// bkn: the bootstrapping key to use (NULL: the context's); with keytab non-NULL gate g uses
// keytab[kid[g]] instead (device arrays). The matrix-core forms (waves 32 and 33) need the
// context's own key and a workspace of mf_work_bytes(B, trlwe == NULL) bytes in mf_work;
// without them the best NTT form for B runs instead.
// tile_mfkeys (device, one pointer per tile of MF_TILE gates, NULL for none): the byte-plane
// key of each tile's key set, for batches whose key-set ranges start on tile boundaries; with
// it the matrix-core forms also run batches of other key sets.
hipError_t launch_blind_rotate(const vsp_context* ctx, const uint8_t* ops, const uint32_t* abar, uint32_t* tlwe1,
                               uint32_t* trlwe, uint64_t B, int waves, hipStream_t st, const uint64_t* bkn = nullptr,
                               const uint64_t* const* keytab = nullptr, const uint16_t* kid = nullptr,
                               void* mf_work = nullptr, bool instrument = false,
                               const int8_t* const* tile_mfkeys = nullptr);
// Matrix-core form (blind_rotate_mfma.hip): key bytes, workspace bytes, key conversion from
// the torus key [n][2l][2][N] on the device, and the launch sequence.
hipError_t init_mf_kernel_attributes();
size_t mf_key_bytes();
size_t mf_work_bytes(uint64_t B, bool need_acc);
hipError_t launch_mf_key(const uint32_t* bk, int8_t* E, hipStream_t st);
// Matrix-core key switch (keyswitch_mfma.hip).
size_t ks_mf_key_bytes();
hipError_t launch_ks_mfkey(const uint32_t* ksk, int8_t* KB, hipStream_t st);
hipError_t launch_keyswitch_mfma(const int8_t* KB, const uint8_t* ops, const uint32_t* tlwe1, const uint32_t* idxo,
                                 uint32_t* out, uint64_t B, hipStream_t st);
// Split form (waves 33): two launches per step, `groups` (kSplitGroupChoices) workgroups per
// (tile, output, sub-product); same workspace as the fused form.
hipError_t launch_blind_rotate_mfsplit(const vsp_context* ctx, const uint8_t* ops, const uint32_t* abar,
                                       uint32_t* tlwe1, uint32_t* trlwe, uint64_t B, void* work, int groups,
                                       hipStream_t st, bool instrument = false,
                                       const int8_t* const* tkeys = nullptr);
// With instrument set (eager calls from the caller's thread only), one event pair of class 3
// brackets the step launches.
hipError_t launch_blind_rotate_mfma(const vsp_context* ctx, const uint8_t* ops, const uint32_t* abar, uint32_t* tlwe1,
                                    uint32_t* trlwe, uint64_t B, void* work, hipStream_t st, bool instrument = false,
                                    const int8_t* const* tkeys = nullptr);
// Identity key switch TLWE1 [B][N+1] -> TLWE0 [B][n+1] (outputs scattered by idxo if given).
// form: 0 one workgroup per gate, 1 row-stationary tiles, 2 LDS-staged split, 3 matrix cores
// (the context's own key only; other keys run form 2), -1 the tuned one.
constexpr int kKsForms = 4;
// ksk: the key-switching key to use (NULL: the context's); ks_mf: its byte-plane form (needed
// for form 3 with a key other than the context's).
hipError_t launch_keyswitch(const vsp_context* ctx, const uint8_t* ops, const uint32_t* tlwe1, const uint32_t* idxo,
                            uint32_t* out, uint64_t B, hipStream_t st, int form = -1, const uint32_t* ksk = nullptr,
                            const int8_t* ks_mf = nullptr);
// out[j] = C_j (ext) x_j, or with `x0` given: out[j] = x0_j + C_j (ext) (x_j - x0_j).
hipError_t launch_ext_product(const vsp_context* ctx, const uint64_t* Cn, const uint32_t* x, uint32_t* out,
                              uint64_t J, hipStream_t st);
hipError_t launch_polymul(const vsp_context* ctx, const int32_t* a, const uint32_t* b, uint32_t* out, uint64_t J,
                          hipStream_t st);

// ---------------------------------------------------------------- circuits (circuit.hip)
// Launches every level of a circuit on `st` (eager or under capture); the circuit's own wire
// buffer [inputs + gates][n+1].
hipError_t circuit_launch_levels(vsp_circuit* c, hipStream_t st);
uint32_t* circuit_wires(vsp_circuit* c);

// ---------------------------------------------------------------- CMUX memory (memory.hip)
// Sets the LDS limits of the CMUX kernels (once per process and device, before any launch).
hipError_t init_memory_kernel_attributes();
// One level of CMUX trees: for r < R, blk < nb, m < W/2:
//   out[(r nb + blk) W/2 + m] = CMUX(sel[r * sel_r_stride + selbit], in[r s_r + blk s_b + 2m], in[.. + 2m + 1]).
hipError_t launch_cmux_tree_level(const vsp_context* ctx, const uint64_t* sel, uint64_t sel_r_stride, int selbit,
                                  const uint32_t* in, uint64_t s_r, uint64_t s_b, uint32_t* out, uint64_t R,
                                  uint64_t nb, uint64_t W, hipStream_t st);
// R <- CMUX(C_j, R, X^{-w 2^j} R) for j < rotbits, per read.
hipError_t launch_rom_rotate(const vsp_context* ctx, const uint64_t* sel, uint64_t sel_r_stride, uint32_t* acc,
                             uint64_t R, int rotbits, int w, hipStream_t st);
// SampleExtract_h for h < W of each TRLWE: in [R][2][N] -> out [R][W][N+1].
hipError_t launch_sample_extract(const uint32_t* in, uint32_t* out, uint64_t R, int W, hipStream_t st);
// u_i = acc_and[i] + acc_andnot[i] + (0, mu X^0).
hipError_t launch_ram_control(const uint32_t* acc2, uint32_t* u, int w, hipStream_t st);
// Write bars: SE_0 of the chained CMUX per (bit i, address A) into tlwe1 [w 2^v][N+1].
hipError_t launch_ram_bars(const vsp_context* ctx, const uint64_t* sel, const uint64_t* selneg, const uint32_t* ram,
                           const uint32_t* u, uint32_t* tlwe1, int v, int w, hipStream_t st);
// out = G - C for TRGSW [count][2l][2][N] (torus), the comparison with a constant 0 bit.
hipError_t launch_gadget_minus(const uint32_t* C, uint32_t* out, uint64_t count, hipStream_t st);

}  // namespace vsp
