/*
 * libvsp: TFHE gate bootstrapping and CMUX memory on one AMD Instinct MI355X (gfx950).
 *
 * The operations are those the server evaluates in "Virtual Secure Platform: A Five-Stage
 * Pipeline Processor over TFHE" (arXiv 2010.09410): homomorphic gates over TLWE ciphertexts
 * (Sec. 2.1.2, "Homomorphic Gates", "Bootstrapping in TFHE") and CMUX-Memory reads and writes
 * (Sec. 8). The caller (the server party) holds the public bootstrapping key; secret keys
 * never reach this library.
 *
 * Conventions used by every call:
 *  - Torus elements are uint32_t (the torus R/Z at resolution 2^-32; arithmetic mod 2^32).
 *  - Parameters are fixed at n = 630, N = 1024, k = 1, l = 3, Bg = 2^6, key switch t = 8,
 *    base 2^2; vsp_context_create rejects anything else with VSP_E_PARAMS.
 *  - TLWE (level 0): n + 1 words (a[0..n-1], b). TLWE (level 1): N + 1 words.
 *    TRLWE: [2][N] (a, then b). TRGSW: [2l][2][N], rows as in Sec. 2.1.2 (rows 0..l-1 carry
 *    m/Bg^j in a, rows l..2l-1 in b).
 *  - Messages are encoded as +-1/8 (bit m -> mu(2m - 1), mu = 1/8), Sec. 2.1.2.
 *  - Pointers named d_* are device memory on the context's device, owned by the caller,
 *    4-byte aligned, and must cover the sizes stated. Pointers named h_* are host memory.
 *    The library never frees caller memory. Outputs must not overlap inputs unless a
 *    call says otherwise (VSP_E_ARG).
 *  - Calls that take a stream validate their arguments synchronously, then enqueue work
 *    asynchronously on that stream (a hipStream_t; NULL = the default stream) and return.
 *    Results are valid after the stream is synchronised. Failures of enqueued work surface
 *    as VSP_E_HIP from a later call or from vsp_context_sync.
 *  - A context is not re-entrant: calls on one context must be ordered by the caller
 *    (one host thread, one stream, or explicit synchronisation). The server serialises
 *    its own work. Circuits, servers and key sets hold a pointer to their context: destroy
 *    them before the context.
 *  - Every call returns a vsp_status; nothing unwinds across this interface. The detail
 *    of the last failure on the calling thread is available from vsp_last_error().
 */
#ifndef VSP_H
#define VSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vsp_status;
#define VSP_OK 0
#define VSP_E_ARG (-1)      /* null / misaligned / undersized / overlapping / out-of-range argument */
#define VSP_E_PARAMS (-2)   /* parameter set differs from the compiled one */
#define VSP_E_NOMEM (-3)    /* device allocation failed */
#define VSP_E_HIP (-4)      /* HIP runtime or kernel failure */
#define VSP_E_STATE (-5)    /* object in the wrong state (e.g. destroyed server, unknown ticket) */
#define VSP_E_CAPACITY (-6) /* server admission refused: request larger than the memory budget */

typedef struct vsp_params {
  uint32_t n, N, k, l, bg_bits, ks_t, ks_basebit;
} vsp_params;

/* Gate opcodes. The linear combinations are the standard TFHE ones on the +-1/8 encoding;
 * NOT negates its first input and needs no bootstrap (Sec. 2.1.2 "Homomorphic Gates"). */
typedef enum vsp_gate {
  VSP_NAND = 0, VSP_AND = 1, VSP_OR = 2, VSP_NOR = 3, VSP_XOR = 4, VSP_XNOR = 5,
  VSP_ANDNOT = 6, /* in0 AND NOT in1 */
  VSP_ORNOT = 7,  /* in0 OR NOT in1 */
  VSP_NOT = 8
} vsp_gate;

/* Launch modes of vsp_gates. */
#define VSP_BATCHED 0  /* all gates of the call in one launch sequence */
#define VSP_PER_GATE 1 /* one launch sequence per gate, serialised on the stream */

typedef struct vsp_context vsp_context;
typedef struct vsp_circuit vsp_circuit;
typedef struct vsp_server vsp_server;
typedef struct vsp_keyset vsp_keyset;
typedef struct vsp_machine vsp_machine;
typedef struct vsp_cbkey vsp_cbkey;

/* A gate of a circuit: opcode and the wire ids of its inputs (in1 ignored by NOT). Wires
 * 0..ninputs-1 are the circuit inputs; gate g writes wire ninputs + g. */
typedef struct vsp_gate_desc {
  uint32_t op, in0, in1;
} vsp_gate_desc;

/* Static text of a status code. */
const char* vsp_status_str(vsp_status s);

/* Detail of the last failure on the calling thread ("" if none). */
const char* vsp_last_error(void);

/* Create a context on HIP device `device`: validates params, uploads the bootstrapping key
 * bk_host [n][2l][2][N] (BK[i] = TRGSW_{s1}(s0[i]), Sec. 2.1.2 "Bootstrapping Key") and the
 * key-switching key ksk_host [N][t][base-1][n+1] (entry [j][p][v-1] = TLWE_{s0}(v s1[j] /
 * base^(p+1))), converts the bootstrapping key to the NTT domain and to the byte-plane forms
 * of the matrix-core blind rotation and key switch on the device (about 330 MB of device
 * memory in all: 62 MB NTT-domain, 98 MB byte-plane and 84 MB key-switch byte-plane forms, and
 * the 83 MB key-switching key), and returns it in *out. Host arrays are copied; the caller keeps them.
 * Synchronous. */
vsp_status vsp_context_create(const vsp_params* params, const uint32_t* bk_host, const uint32_t* ksk_host,
                              int device, vsp_context** out);

/* Destroy a context (waits for its device work first). NULL is accepted. */
vsp_status vsp_context_destroy(vsp_context* ctx);

/* Wait for all work the context enqueued and report any device-side failure. */
vsp_status vsp_context_sync(vsp_context* ctx);

/* Homomorphic gates (Sec. 2.1.2 "Homomorphic Gates"; the paper's processor evaluates one
 * per netlist gate, Sec. 2.3): for g < B, d_out[g] = op_g(d_in0[g], d_in1[g]) where each
 * non-NOT gate is linear combination -> modulus switch -> blind rotation (n CMUX external
 * products) -> SampleExtract -> identity key switch, giving a fresh TLWE of the gate's
 * output bit. d_ops [B] (uint8, vsp_gate codes; an invalid code yields an all-zero output
 * and is reported by vsp_context_sync), d_in0, d_in1, d_out [B][n+1]. B = 0 is a no-op.
 * mode: VSP_BATCHED or VSP_PER_GATE (same results, bit for bit). */
vsp_status vsp_gates(vsp_context* ctx, const uint8_t* d_ops, const uint32_t* d_in0, const uint32_t* d_in1,
                     uint32_t* d_out, uint64_t B, int mode, void* stream);

/* vsp_gates without any device allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). Same arguments,
 * results and errors as vsp_gates, bit for bit, with B <= 2048 (larger B: VSP_E_ARG, nothing
 * enqueued). The intermediate ciphertexts live in one fixed 13.6 MB device array per GPU
 * (2048 modulus-switched inputs and 2048 extracted TLWE rows), held until the process ends;
 * the blind rotation runs in its NTT forms (the matrix-core form needs a larger workspace).
 * Every call on one GPU shares that array, so calls that overlap on a GPU (other streams,
 * other contexts or threads) race and must be ordered by the caller. */
vsp_status vsp_gates_noalloc(vsp_context* ctx, const uint8_t* d_ops, const uint32_t* d_in0, const uint32_t* d_in1,
                             uint32_t* d_out, uint64_t B, int mode, void* stream);

/* Gate bootstrapping with the bootstrapping key read from per-gate copies: the measurement of
 * what key reuse contributes to the batched path. The paper's gate evaluation engine hands
 * each gate to a worker as a task of its own (Sec. 6.2(d), list scheduling), so every gate's
 * bootstrap makes its own pass over the key; a batch here shares one pass among all its gates
 * (Sec. 2.3: gates of one level are independent). Same results as vsp_gates in batched mode, bit for bit, with
 * the blind rotation in the NTT form `waves` (3, 4 or 8) and gate g reading device copy
 * g mod `copies` of the converted key: once `copies` reaches the number of gates the form
 * holds at once, no two resident gates read the same key bytes and nothing of the key is
 * reused through the caches; copies = 1 is the ordinary shared key. 1 <= copies <= 65536,
 * B <= 2^22; *br_ms receives the blind rotation's time (HIP events on `stream`). Allocates
 * copies x 61.9 MB (copies > 1) for the duration of the call (VSP_E_NOMEM when the device
 * lacks it, nothing enqueued) and returns only after the stream has drained. */
vsp_status vsp_gates_key_copies(vsp_context* ctx, const uint8_t* d_ops, const uint32_t* d_in0, const uint32_t* d_in1,
                                uint32_t* d_out, uint64_t B, int waves, uint32_t copies, void* stream,
                                double* br_ms);

/* Bootstrapping that returns a TRLWE (Sec. 2.1.2 "Bootstrapping in TFHE", without SE and
 * IKS): d_out[g] [2][N] is the blind-rotation accumulator of op_g(in0, in1) with the test
 * vector mu in every coefficient (constant coefficient encodes the gate's output bit).
 * NOT is rejected (VSP_E_ARG is reported by vsp_context_sync as an invalid op). */
vsp_status vsp_bootstrap_trlwe(vsp_context* ctx, const uint8_t* d_ops, const uint32_t* d_in0,
                               const uint32_t* d_in1, uint32_t* d_out, uint64_t B, void* stream);

/* Levelled circuit (the gate-evaluation engine's per-cycle work, Sec. 6.2(d)): gates
 * [ngates] must be in topological order (each input wire id below the gate's own wire).
 * Levelises, plans one batched launch per level and captures the level sequence in a HIP
 * graph. Synchronous. */
vsp_status vsp_circuit_create(vsp_context* ctx, const vsp_gate_desc* gates, uint64_t ngates, uint64_t ninputs,
                              vsp_circuit** out);

/* Evaluate the circuit: d_inputs [ninputs][n+1] -> d_wires [ninputs + ngates][n+1] (all
 * wires, inputs first). Replays the captured graph on `stream`. */
vsp_status vsp_circuit_run(vsp_circuit* c, const uint32_t* d_inputs, uint32_t* d_wires, void* stream);

/* Same evaluation launching each level eagerly (no graph), recording the device time of
 * every level into h_level_ms [nlevels] (synchronises the stream). */
vsp_status vsp_circuit_run_timed(vsp_circuit* c, const uint32_t* d_inputs, uint32_t* d_wires, void* stream,
                                 float* h_level_ms);

/* Number of levels of the circuit and the width of its widest level. */
vsp_status vsp_circuit_info(const vsp_circuit* c, uint64_t* nlevels, uint64_t* max_width);
vsp_status vsp_circuit_destroy(vsp_circuit* c);

/* ROM read by CMUX tree over packed TRLWE cells (Sec. 8.3: LUT with vertical and
 * horizontal packing). d_rom [P][2][N]: P = 2^(v - log2(N / w)) cells; coefficient w*q + b
 * of cell h holds bit b of word (N/w)*h + q. d_addr [R][v][2l][2][N]: per read, TRGSW
 * encryptions of the v address bits, least significant first. The high v - log2(N/w) bits
 * walk a CMUX tree over the cells, the low log2(N/w) bits rotate the chosen cell by
 * X^(-w q) with CMUXes, then bit b is KS(SampleExtract_b). d_out [R][w][n+1]. w must divide
 * N, be a power of two and P >= 1; R w <= 2^22. */
vsp_status vsp_rom_read(vsp_context* ctx, const uint32_t* d_rom, uint32_t P, const uint32_t* d_addr, uint32_t v,
                        uint32_t w, uint32_t* d_out, uint64_t R, void* stream);

/* RAM read unit (Sec. 8.2): d_ram [w][2^v][2][N], block i holds bit i of every word in its
 * constant coefficient. Per read and bit: CMUX tree over the 2^v cells (address bit d
 * selects at level d, least significant first), SampleExtract_0, key switch.
 * d_addr [R][v][2l][2][N]; d_out [R][w][n+1]. 1 <= v <= 16, 1 <= w <= 1024, R w <= 2^22. */
vsp_status vsp_ram_read(vsp_context* ctx, const uint32_t* d_ram, uint32_t v, uint32_t w, const uint32_t* d_addr,
                        uint32_t* d_out, uint64_t R, void* stream);

/* RAM write (Sec. 8.2, read unit + control unit + write unit): with r_i the read of bit i
 * at the address, the control unit forms u_i = BR(AND(f, x_i)) + BR(ANDNOT(r_i, f)) +
 * (0, mu X^0) (HomMUX without SE and IKS); each of the w 2^v write bars (bit i, address A)
 * chains v CMUXes y <- CMUX(s_d, R[i][A], y) from y = u_i, with s_d = C_d when bit d of A is
 * 1 and G - C_d otherwise (Sec. 8.2 Remark), and refreshes R[i][A] <- BR(KS(SE_0(y))).
 * d_ram is updated in place; d_addr [v][2l][2][N]; d_flag [n+1]; d_data [w][n+1].
 * 1 <= v <= 16, 1 <= w <= 1024, w 2^v <= 2^22. */
vsp_status vsp_ram_write(vsp_context* ctx, uint32_t* d_ram, uint32_t v, uint32_t w, const uint32_t* d_addr,
                         const uint32_t* d_flag, const uint32_t* d_data, void* stream);

/* A clocked circuit (the cycle loop of the paper's evaluation engine, Sec. 6.2(d)): wires
 * 0..ninputs-1 are the external inputs of a cycle, ninputs..ninputs+nstate-1 the flip-flop
 * outputs, and gate g writes wire ninputs + nstate + g (gates as for vsp_circuit_create,
 * reading any earlier wire). At the end of every cycle flip-flop k latches wire
 * next_state[k] (any wire; all flip-flops latch at once). The level sequence and the latch
 * are captured once in a HIP graph. */
vsp_status vsp_machine_create(vsp_context* ctx, const vsp_gate_desc* gates, uint64_t ngates, uint64_t ninputs,
                              uint64_t nstate, const uint32_t* next_state, vsp_machine** out);

/* Runs ncycles clock cycles on `stream`: d_state [nstate][n+1] holds the flip-flops' state
 * before (in) and after (out) the run; d_inputs [ncycles][ninputs][n+1] the external inputs
 * of every cycle (NULL when ninputs = 0); d_wires (optional, NULL to skip) receives all
 * [ninputs + nstate + ngates][n+1] wires of the last cycle, whose flip-flop rows already hold
 * the latched state. A machine runs one call at a time. */
vsp_status vsp_machine_run(vsp_machine* m, const uint32_t* d_inputs, uint32_t* d_state, uint32_t* d_wires,
                           uint64_t ncycles, void* stream);
vsp_status vsp_machine_destroy(vsp_machine* m);

/* Give a machine a one-cycle single-port RAM (the CMUX memory of Sec. 8.2, fed by the
 * processor's wires as TLWE): d_ram [w][2^v][2][N] holds its cells (caller's device memory,
 * updated in place by every cycle's write). Each cycle, after the DAG, the wires
 * addr_wires[0..v) (address, least significant bit first), flag_wire (write flag) and
 * data_wires[0..w) (write data) are staged; circuit bootstrapping turns the address bits into
 * TRGSW selectors (key: vsp_cbkey_create); the RAM is read at that address (contents before
 * the write) into flip-flops read_state[0..w) (their next_state entries are then ignored);
 * and the write of vsp_ram_write runs with the staged flag and data. Wire ids as for
 * vsp_machine_create (0..ninputs-1 inputs, then flip-flops, then gates). One RAM per machine
 * (VSP_E_STATE for a second); the key and d_ram must outlive the machine. */
vsp_status vsp_machine_attach_ram(vsp_machine* m, vsp_cbkey* key, uint32_t* d_ram, uint32_t v, uint32_t w,
                                  const uint32_t* addr_wires, uint32_t flag_wire, const uint32_t* data_wires,
                                  const uint32_t* read_state);

/* Continuous-batching server over one context (Bob evaluating many clients' circuits,
 * Sec. 4.1): admits submitted circuits while their resident wire buffers fit in
 * mem_budget_bytes of device memory, and each iteration launches one batch of ready
 * gates taken across all admitted circuits (at most max_batch gates). Runs its own host
 * thread and stream. */
vsp_status vsp_server_create(vsp_context* ctx, uint64_t mem_budget_bytes, uint64_t max_batch, vsp_server** out);

/* Submit a circuit (gates as for vsp_circuit_create) with host inputs h_inputs
 * [ninputs][n+1]; returns a ticket. VSP_E_CAPACITY if the circuit alone exceeds the
 * memory budget. The input array is copied before the call returns. */
vsp_status vsp_server_submit(vsp_server* s, const vsp_gate_desc* gates, uint64_t ngates, uint64_t ninputs,
                             const uint32_t* h_inputs, uint64_t* ticket);

/* Poll a ticket: *done = 1 once finished, and then (if h_wires is not NULL) copies all
 * wires [ninputs + ngates][n+1] to h_wires and releases the ticket; latency_ms (if not
 * NULL) receives submit-to-completion time. *done = 0 while queued or running. */
vsp_status vsp_server_poll(vsp_server* s, uint64_t ticket, uint32_t* h_wires, int* done, double* latency_ms);

/* A further client's key set on the context's GPU (the protocol gives every client its own
 * keys, Sec. 4.1): bk_host [n][2l][2][N] and ksk_host [N][t][base-1][n+1] as for
 * vsp_context_create, converted and copied to the device in the same forms (about 330 MB); the
 * caller keeps its arrays. Synchronous. A key set must outlive every request submitted with it. */
vsp_status vsp_keyset_create(vsp_context* ctx, const uint32_t* bk_host, const uint32_t* ksk_host, vsp_keyset** out);
vsp_status vsp_keyset_destroy(vsp_keyset* k);

/* vsp_server_submit for a circuit encrypted under `keys` (a key set of the server's context;
 * NULL means the context's own keys). A batch may hold the ready gates of up to 64 key sets:
 * it is ordered by key set, each gate's blind rotation reads its own key, and the key switch
 * runs once per key set. */
vsp_status vsp_server_submit_keyset(vsp_server* s, const vsp_keyset* keys, const vsp_gate_desc* gates,
                                    uint64_t ngates, uint64_t ninputs, const uint32_t* h_inputs, uint64_t* ticket);

/* Counters: gates launched, batches launched, peak resident bytes. */
vsp_status vsp_server_stats(vsp_server* s, uint64_t* gates, uint64_t* batches, uint64_t* peak_bytes);

/* Stop the server thread (finishing admitted work) and free it. NULL is accepted. */
vsp_status vsp_server_destroy(vsp_server* s);

/* Homomorphic MUX of B rows (the three-operand gate of Sec. 2.1.2): d_out[g] = d_sel[g] ? d_in1[g]
 * : d_in0[g] on encrypted bits, all [B][n+1] TLWE rows under the LWE key. Each MUX bootstraps
 * AND(s, c1) and ANDNOT(c0, s) to TRLWE, adds them and (0, mu) (the HomMUX without SE and IKS
 * of Sec. 2.1.2, as in the RAM control unit of Sec. 8.2), then SampleExtracts and key-switches
 * once: twice a gate's blind rotations, one key switch. d_out must not overlap the inputs
 * (VSP_E_ARG). Asynchronous on `stream`. */
vsp_status vsp_mux(vsp_context* ctx, const uint32_t* d_sel, const uint32_t* d_in1, const uint32_t* d_in0,
                   uint32_t* d_out, uint64_t B, void* stream);

/* Autotuner for the batched launches (the level executor's tile and batch shapes). A gate's
 * blind rotation runs on one wave (or, in the latency shape, on three waves that split each
 * external product by gadget level), so a batch of B gates runs in ceil(B / cap) rounds, cap
 * being the gates the GPU holds at once for a workgroup shape (4 or 8 gates per workgroup, or
 * one gate per three-wave workgroup). The matrix-core form (32) instead runs each step as int8
 * MFMA products of the batch's digit rows with the key's Toeplitz blocks (tiles of 32 gates;
 * one round holds 16 gates per compute unit; used by vsp_gates and vsp_bootstrap_trlwe with the
 * context's own key, the other callers run the 8-gate form in its place; it needs a workspace
 * of 26 KiB per gate (18 KiB when the output is the TRLWE accumulator), grown on demand). This call times one full round of each shape on random
 * ciphertexts, and times the four key-switch forms (0: one workgroup per gate gathering its
 * key rows; 1: tiles of 16 gates reading each key row once and selecting in registers;
 * 2: tiles of 16 gates staging key rows through LDS, with the j range split over workgroups
 * and atomic accumulation; 3: int8 MFMA products of one-hot digit rows with the key's byte
 * planes, for the context's own key, other keys running form 2) for each batch-size bucket up
 * to max_batch (buckets end at 1, 16,
 * 64, 256, 1024, 2048, 4096 gates; larger batches share the last). Every candidate must give
 * bit-identical outputs (else VSP_E_HIP). Later launches pick the shape with the fewest
 * rounds x round time, and the faster key switch for their bucket. With cache_path non-NULL
 * the measurements are read from that JSON file when it holds an entry for this GPU, and
 * otherwise measured and written there. Synchronous; allocates and frees its own buffers. */
vsp_status vsp_autotune(vsp_context* ctx, uint64_t max_batch, const char* cache_path);

/* The launch choice for a batch of B gates: *br_waves (4 or 8 gates per workgroup at one wave
 * per gate, 3 for one gate per workgroup on three waves, 32 for the matrix-core form),
 * *ks_form (0, 1, 2 or 3). Before vsp_autotune (or after it returned a bucket to the model),
 * the blind-rotation shape comes from the round-time model with default round times, and the
 * key switch is form 2 up to 256 gates and form 3 above. */
vsp_status vsp_tuning_get(const vsp_context* ctx, uint64_t B, int* br_waves, int* ks_form);

/* Pin the launch choice for the bucket containing B: br_waves 3, 4, 8 or 32 (0 returns that
 * bucket to the round-time model), ks_form 0, 1, 2 or 3. Results are the same for every choice. */
vsp_status vsp_tuning_set(vsp_context* ctx, uint64_t B, int br_waves, int ks_form);

/* Pin how the split matrix-core form (the blind rotation's form 33) cuts a step at the timed
 * batch size that covers B (1, 16, 64, 256, 512, 768, 1024, 1280, 1536, 1792, 2048, 3072,
 * 4096 gates; batches up to that size and above the previous one use it): groups = 1, 2, 3
 * or 6 groups of TRGSW rows per (tile, output, sub-product), 12 or 24 for one row per
 * workgroup and the four byte planes in 2 or 4 ranges (shares added with integer atomics);
 * -1, -2, -3 or -6 for those row groups with the shares stored as partial sums that the next
 * digit launch adds up (batches above 3,072 gates fall back to atomics); 0 for the count that
 * fills the chip.
 * *previous (may be NULL) receives the value it replaces. Results are the same for every
 * choice; vsp_autotune overwrites the setting. */
vsp_status vsp_tuning_set_split(vsp_context* ctx, uint64_t B, int groups, int* previous);

/* Kernel-time instrumentation (for benchmarks): with on >= 1, the blind-rotation, key-switch
 * and gate-prologue launches made by vsp_gates / vsp_bootstrap_trlwe / vsp_mux on the calling
 * thread are bracketed by HIP events on the stream they run on; for the matrix-core form one
 * more event pair brackets the whole sequence of its 630 step launches. Every call with
 * on = 1, every on-th call of each kind with on > 1. Launches under stream capture, from
 * circuits, memory calls and the server are never instrumented. on = 0 disables, on < 0 is
 * VSP_E_ARG. Enabling resets the totals. */
vsp_status vsp_profile_enable(vsp_context* ctx, int on);

/* Device time (ms, summed) and number of kernel launches it covers, for kernel `which` since
 * enabling: 0 = blind rotation, 1 = key switch, 2 = gate prologue, 3 = step kernel of the
 * matrix-core blind rotation (630 launches per bracketed sequence, so total / launches is the
 * average step launch including the gaps between launches). Synchronises the device. */
vsp_status vsp_profile_read(vsp_context* ctx, int which, double* total_ms, uint64_t* launches);

/* Measurement entry: the device's throughput of the arithmetic modulo the NTT prime
 * p = 2^64 - 2^32 + 1 that the transform-domain blind rotation is built from (the polynomial
 * products of the external product, Sec. 2.1.2, computed by NTT over the prime of Sec. 6.2(a)):
 * general products and lazy sums mod p, each in independent register-resident chains at full
 * occupancy with `iters` operations per chain (16 <= iters <= 2^24), timed with HIP events.
 * Writes operations per second to *mulmod_per_s and *addmod_per_s. Allocates and frees its
 * own small buffers and synchronises the device; VSP_E_ARG for NULL outputs, a bad device
 * or iters out of range. */
vsp_status vsp_measure_modp(int device, uint32_t iters, double* mulmod_per_s, double* addmod_per_s);

/* Test entry: d_out[j] = C_j (ext) x_j for J (TRGSW, TRLWE) pairs, the external product
 * at the heart of CMUX (Sec. 2.1.2 "CMUX"). d_trgsw [J][2l][2][N], d_x and d_out [J][2][N]. */
vsp_status vsp_debug_external_product(vsp_context* ctx, const uint32_t* d_trgsw, const uint32_t* d_x,
                                      uint32_t* d_out, uint64_t J, void* stream);

/* Test entry: d_out[j] = d_a[j] * d_b[j] in Z[X]/(X^N+1) mod 2^32 through the NTT path.
 * d_a holds small signed integers (|a| <= 2^20, so every exact coefficient stays below
 * p/2); d_b torus values. Arrays [J][N]. */
vsp_status vsp_debug_polymul(vsp_context* ctx, const int32_t* d_a, const uint32_t* d_b, uint32_t* d_out,
                             uint64_t J, void* stream);

/* ---------------------------------------------------------------- circuit bootstrapping
 * TLWE -> TRGSW (Sec. 2.1.2 "Circuit Bootstrapping"), the conversion the CMUX memory applies
 * to its address bits (Sec. 8.2). The paper fixes no parameters for it; this library reads
 * them as a level-2 ring of degree N2 = 2048 over the 2^64 torus with an l2 = 4 x 2^9 gadget
 * and private functional key switching to level-1 TRLWE with t2 = 12 digits of 2 bits.
 *
 * vsp_cbkey_create uploads the level-2 bootstrapping key bk2_host [n][2 l2][2][N2] (uint64
 * torus words; BK2[i] = TRGSW2_{s2}(s0[i]), rows as the level-1 TRGSW) and the two private
 * key-switching keys pksk_host [2][N2+1][t2][3][2][N] (uint32; entry [u][k][p][v-1] is a
 * level-1 TRLWE of f_u(v z_k / 4^(p+1)) with z = (-s2[0..N2-1], 1), f_0(x) = -s1 x and
 * f_1(x) = x), converts the first to its transformed layout on the device (about 645 MB; the
 * second takes 1.2 GB) and returns the key in *out. Host arrays are copied. Synchronous.
 * Destroy it before its context. */
vsp_status vsp_cbkey_create(vsp_context* ctx, const uint64_t* bk2_host, const uint32_t* pksk_host, vsp_cbkey** out);
vsp_status vsp_cbkey_destroy(vsp_cbkey* key);

/* The level-2 blind rotation's form for later vsp_circuit_bootstrap calls with this key: 0 (the
 * default) picks by batch size, 1 forces one workgroup of four waves per (conversion, gadget
 * level) job, two per compute unit (throughput), 2 forces eight waves per job, one per compute
 * unit, with a step's eight digit rows transformed at once (latency). Results are the same
 * for every form; form outside [0, 2] is VSP_E_ARG. */
vsp_status vsp_cbkey_set_form(vsp_cbkey* key, int form);

/* d_out[r] [2l][2][N] = the level-1 TRGSW of the bit that the level-0 TLWE d_in[r] [n+1]
 * encrypts (+-1/8 encoding), for r < R: for each gadget level j = 1..l a level-2 blind
 * rotation with test vector 1/(2 Bg^j), SampleExtract at 0 plus 1/(2 Bg^j), then the two
 * private key switches, giving rows j-1 (f_0) and l+j-1 (f_1). The output is usable as a
 * selector of vsp_rom_read / vsp_ram_read / vsp_ram_write. R = 0 is a no-op; R above 2^20 is
 * VSP_E_ARG. The key's scratch grows on demand (allocation). */
vsp_status vsp_circuit_bootstrap(vsp_context* ctx, vsp_cbkey* key, const uint32_t* d_in, uint32_t* d_out,
                                 uint64_t R, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VSP_H */
