// Clocked circuits: the cycle loop of the paper's evaluation engine (Sec. 6.2(d)), which
// splits a processor netlist into a combinational DAG and flip-flops and evaluates the DAG
// once per clock. A machine is a levelled circuit whose inputs are the cycle's external
// inputs followed by the flip-flop outputs; after the DAG, every flip-flop latches the wire
// named for it. One HIP graph per machine holds the level sequence and the latch, and each
// cycle replays it. A machine can also hold a RAM (the CMUX memory of Sec. 8.2): each cycle
// its address, write-flag and write-data wires are staged inside the graph before the latch,
// then the address bits are circuit-bootstrapped to TRGSW selectors, the RAM is read into
// the flip-flops named for the read port, and written under the flag.
#include <vector>

#include "vsp_internal.h"

using namespace vsp;

struct vsp_machine {
  vsp_context* ctx = nullptr;
  vsp_circuit* circ = nullptr;
  uint64_t ngates = 0, ninputs = 0, nstate = 0;
  uint32_t* d_next = nullptr;   // [nstate] wire id latched into flip-flop k
  uint32_t* d_latch = nullptr;  // [nstate][n+1] staging of the next state
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // RAM port (optional)
  vsp_cbkey* cbkey = nullptr;
  uint32_t* d_ram = nullptr;       // caller's cells [w][2^v][2][N]
  uint32_t v = 0, w = 0;
  uint32_t* d_memidx = nullptr;    // [v + 1 + w] wire ids: address bits, write flag, write data
  uint32_t* d_memstage = nullptr;  // [v + 1 + w][n+1] their values in the cycle
  uint32_t* d_sel = nullptr;       // [v][2l][2][N] selectors from circuit bootstrapping
  uint32_t* d_rd = nullptr;        // [w][n+1] read data
  uint32_t* d_rdrow = nullptr;     // [w] wire rows of the read-port flip-flops
};

namespace {

constexpr size_t T0B = (LWE_N + 1) * 4;

// stage[k] = wires[next[k]] for every flip-flop (all reads before any flip-flop row changes).
__global__ __launch_bounds__(256) void k_latch_gather(const uint32_t* __restrict__ wires,
                                                      const uint32_t* __restrict__ next, uint32_t* __restrict__ stage,
                                                      uint64_t nstate) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nstate * (LWE_N + 1)) return;
  const uint64_t k = i / (LWE_N + 1);
  const uint64_t c = i - k * (LWE_N + 1);
  stage[i] = wires[(uint64_t)next[k] * (LWE_N + 1) + c];
}

// dst rows rows[k] (stride n+1) = src[k] for k < count.
__global__ __launch_bounds__(256) void k_scatter_rows(uint32_t* __restrict__ dst, const uint32_t* __restrict__ rows,
                                                      const uint32_t* __restrict__ src, uint64_t count) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count * (LWE_N + 1)) return;
  const uint64_t k = i / (LWE_N + 1);
  const uint64_t c = i - k * (LWE_N + 1);
  dst[(uint64_t)rows[k] * (LWE_N + 1) + c] = src[i];
}

void free_ram_port(vsp_machine* m) {
  for (void* p : {(void*)m->d_memidx, (void*)m->d_memstage, (void*)m->d_sel, (void*)m->d_rd, (void*)m->d_rdrow})
    if (p) (void)hipFree(p);
  m->d_memidx = m->d_memstage = m->d_sel = m->d_rd = m->d_rdrow = nullptr;
  m->cbkey = nullptr;
  m->d_ram = nullptr;
  m->v = m->w = 0;
}

void free_graph(vsp_machine* m) {
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  m->exec = nullptr;
  m->graph = nullptr;
}

void free_machine(vsp_machine* m) {
  if (!m) return;
  (void)hipSetDevice(m->ctx->device);
  (void)hipDeviceSynchronize();
  free_graph(m);
  if (m->cap) (void)hipStreamDestroy(m->cap);
  for (void* p : {(void*)m->d_next, (void*)m->d_latch})
    if (p) (void)hipFree(p);
  free_ram_port(m);
  if (m->circ) (void)vsp_circuit_destroy(m->circ);
  delete m;
}

// Captures one clock cycle into the machine's graph: the level sequence, the staging of the
// RAM port's wires (if any), then the latch (gather into staging, copy into the flip-flop
// rows).
vsp_status capture_cycle(vsp_machine* m) {
  free_graph(m);
  hipError_t e;
  if ((e = hipStreamBeginCapture(m->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return hip_fail(e, "begin capture");
  hipError_t le = circuit_launch_levels(m->circ, m->cap);
  uint32_t* wires = circuit_wires(m->circ);
  if (le == hipSuccess && m->d_ram) {
    const uint64_t nm = (uint64_t)m->v + 1 + m->w;
    hipLaunchKernelGGL(k_latch_gather, dim3((unsigned)((nm * (LWE_N + 1) + 255) / 256)), dim3(256), 0, m->cap, wires,
                       m->d_memidx, m->d_memstage, nm);
    le = hipGetLastError();
  }
  if (le == hipSuccess && m->nstate) {
    hipLaunchKernelGGL(k_latch_gather, dim3((unsigned)((m->nstate * (LWE_N + 1) + 255) / 256)), dim3(256), 0, m->cap,
                       wires, m->d_next, m->d_latch, m->nstate);
    le = hipGetLastError();
    if (le == hipSuccess)
      le = hipMemcpyAsync(wires + m->ninputs * (LWE_N + 1), m->d_latch, m->nstate * T0B, hipMemcpyDeviceToDevice,
                          m->cap);
  }
  e = hipStreamEndCapture(m->cap, &m->graph);
  if (le != hipSuccess) return hip_fail(le, "cycle launch during capture");
  if (e != hipSuccess) return hip_fail(e, "end capture");
  if ((e = hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0)) != hipSuccess)
    return hip_fail(e, "graph instantiate");
  return VSP_OK;
}

// The RAM port's work of one cycle, after the graph: circuit bootstrapping of the staged
// address bits, the read into the read-port flip-flops, then the write under the flag.
vsp_status ram_port_cycle(vsp_machine* m, hipStream_t st) {
  vsp_context* ctx = m->ctx;
  vsp_status s;
  uint32_t* wires = circuit_wires(m->circ);
  if ((s = vsp_circuit_bootstrap(ctx, m->cbkey, m->d_memstage, m->d_sel, m->v, st))) return s;
  if ((s = vsp_ram_read(ctx, m->d_ram, m->v, m->w, m->d_sel, m->d_rd, 1, st))) return s;
  hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)(((uint64_t)m->w * (LWE_N + 1) + 255) / 256)), dim3(256), 0, st,
                     wires, m->d_rdrow, m->d_rd, (uint64_t)m->w);
  VSP_HIP(hipGetLastError());
  return vsp_ram_write(ctx, m->d_ram, m->v, m->w, m->d_sel, m->d_memstage + (size_t)m->v * (LWE_N + 1),
                       m->d_memstage + (size_t)(m->v + 1) * (LWE_N + 1), st);
}

}  // namespace

extern "C" {

vsp_status vsp_machine_create(vsp_context* ctx, const vsp_gate_desc* gates, uint64_t ngates, uint64_t ninputs,
                              uint64_t nstate, const uint32_t* next_state, vsp_machine** out) {
  if (out == nullptr) return fail(VSP_E_ARG, "out is NULL");
  *out = nullptr;
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  if (nstate > 0 && next_state == nullptr) return fail(VSP_E_ARG, "next_state is NULL");
  if (nstate > kMaxLaunch) return fail(VSP_E_ARG, "too many flip-flops");
  const uint64_t nwires = ninputs + nstate + ngates;
  for (uint64_t k = 0; k < nstate; k++)
    if (next_state[k] >= nwires) return fail(VSP_E_ARG, "flip-flop " + std::to_string(k) + " latches a wire that does not exist");
  auto* m = new vsp_machine();
  m->ctx = ctx;
  m->ngates = ngates;
  m->ninputs = ninputs;
  m->nstate = nstate;
  auto bail = [&](vsp_status s) {
    free_machine(m);
    return s;
  };
  vsp_status s = vsp_circuit_create(ctx, gates, ngates, ninputs + nstate, &m->circ);
  if (s) {
    m->circ = nullptr;
    return bail(s);
  }
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return bail(hip_fail(e, "hipSetDevice"));
  if (nstate) {
    if ((e = hipMalloc(&m->d_next, nstate * 4)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
    if ((e = hipMalloc(&m->d_latch, nstate * T0B)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
    if ((e = hipMemcpy(m->d_next, next_state, nstate * 4, hipMemcpyHostToDevice)) != hipSuccess)
      return bail(hip_fail(e, "upload"));
  }
  // one clock cycle: the level sequence, then the latch (gather into staging, copy into the
  // flip-flop rows)
  if ((e = hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking)) != hipSuccess) return bail(hip_fail(e, "stream"));
  if ((s = capture_cycle(m))) return bail(s);
  *out = m;
  return VSP_OK;
}

vsp_status vsp_machine_attach_ram(vsp_machine* m, vsp_cbkey* key, uint32_t* d_ram, uint32_t v, uint32_t w,
                                  const uint32_t* addr_wires, uint32_t flag_wire, const uint32_t* data_wires,
                                  const uint32_t* read_state) {
  if (m == nullptr) return fail(VSP_E_ARG, "machine is NULL");
  if (key == nullptr) return fail(VSP_E_ARG, "key is NULL");
  if (v < 1 || v > 16 || w < 1 || w > 1024) return fail(VSP_E_ARG, "v must be in [1, 16] and w in [1, 1024]");
  if (((uint64_t)w << v) > kMaxLaunch) return fail(VSP_E_ARG, "w * 2^v must not exceed 2^22");
  if (addr_wires == nullptr || data_wires == nullptr || read_state == nullptr)
    return fail(VSP_E_ARG, "addr_wires, data_wires and read_state must not be NULL");
  if (m->d_ram) return fail(VSP_E_STATE, "the machine already has a RAM");
  const uint64_t nwires = m->ninputs + m->nstate + m->ngates;
  std::vector<uint32_t> idx;
  for (uint32_t b = 0; b < v; b++) idx.push_back(addr_wires[b]);
  idx.push_back(flag_wire);
  for (uint32_t b = 0; b < w; b++) idx.push_back(data_wires[b]);
  for (uint32_t x : idx)
    if (x >= nwires) return fail(VSP_E_ARG, "a RAM port wire does not exist");
  std::vector<uint32_t> rows(w);
  for (uint32_t b = 0; b < w; b++) {
    if (read_state[b] >= m->nstate) return fail(VSP_E_ARG, "a read-port flip-flop does not exist");
    rows[b] = (uint32_t)(m->ninputs + read_state[b]);
  }
  vsp_status s;
  const size_t ram_b = ((size_t)w << v) * 2 * RING_N * 4;
  if ((s = check_device_range(m->ctx, d_ram, ram_b, "d_ram"))) return s;
  VSP_HIP(hipSetDevice(m->ctx->device));
  VSP_HIP(hipDeviceSynchronize());
  m->cbkey = key;
  m->d_ram = d_ram;
  m->v = v;
  m->w = w;
  hipError_t e;
  auto bail = [&](vsp_status st) {
    free_ram_port(m);
    (void)capture_cycle(m);
    return st;
  };
  if ((e = hipMalloc(&m->d_memidx, idx.size() * 4)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
  if ((e = hipMalloc(&m->d_memstage, idx.size() * T0B)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
  if ((e = hipMalloc(&m->d_sel, (size_t)v * 2 * GADGET_L * 2 * RING_N * 4)) != hipSuccess)
    return bail(hip_fail(e, "hipMalloc"));
  if ((e = hipMalloc(&m->d_rd, (size_t)w * T0B)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
  if ((e = hipMalloc(&m->d_rdrow, (size_t)w * 4)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
  if ((e = hipMemcpy(m->d_memidx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(hip_fail(e, "upload"));
  if ((e = hipMemcpy(m->d_rdrow, rows.data(), (size_t)w * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(hip_fail(e, "upload"));
  if ((s = capture_cycle(m))) return bail(s);
  return VSP_OK;
}

vsp_status vsp_machine_run(vsp_machine* m, const uint32_t* d_inputs, uint32_t* d_state, uint32_t* d_wires,
                           uint64_t ncycles, void* stream) {
  if (m == nullptr) return fail(VSP_E_ARG, "machine is NULL");
  vsp_status s;
  const size_t ib = ncycles * m->ninputs * T0B, sb = m->nstate * T0B;
  const size_t wb = (m->ninputs + m->nstate + m->ngates) * T0B;
  if (ib && (s = check_device_range(m->ctx, d_inputs, ib, "d_inputs"))) return s;
  if (sb && (s = check_device_range(m->ctx, d_state, sb, "d_state"))) return s;
  if (d_wires && (s = check_device_range(m->ctx, d_wires, wb, "d_wires"))) return s;
  if (ib && sb && (s = check_no_overlap(d_state, sb, d_inputs, ib, "d_state and d_inputs"))) return s;
  if (d_wires && ib && (s = check_no_overlap(d_wires, wb, d_inputs, ib, "d_wires and d_inputs"))) return s;
  if (d_wires && sb && (s = check_no_overlap(d_wires, wb, d_state, sb, "d_wires and d_state"))) return s;
  VSP_HIP(hipSetDevice(m->ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t* wires = circuit_wires(m->circ);
  if (sb) VSP_HIP(hipMemcpyAsync(wires + m->ninputs * (LWE_N + 1), d_state, sb, hipMemcpyDeviceToDevice, st));
  for (uint64_t c = 0; c < ncycles; c++) {
    if (m->ninputs)
      VSP_HIP(hipMemcpyAsync(wires, d_inputs + c * m->ninputs * (LWE_N + 1), m->ninputs * T0B, hipMemcpyDeviceToDevice,
                             st));
    VSP_HIP(hipGraphLaunch(m->exec, st));
    if (m->d_ram && (s = ram_port_cycle(m, st))) return s;
  }
  if (sb) VSP_HIP(hipMemcpyAsync(d_state, wires + m->ninputs * (LWE_N + 1), sb, hipMemcpyDeviceToDevice, st));
  if (d_wires) VSP_HIP(hipMemcpyAsync(d_wires, wires, wb, hipMemcpyDeviceToDevice, st));
  return VSP_OK;
}

vsp_status vsp_machine_destroy(vsp_machine* m) {
  free_machine(m);
  return VSP_OK;
}

}  // extern "C"
