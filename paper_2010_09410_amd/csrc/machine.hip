// Clocked circuits: the cycle loop of the paper's evaluation engine (Sec. 6.2(d)), which
// splits a processor netlist into a combinational DAG and flip-flops and evaluates the DAG
// once per clock. A machine is a levelled circuit whose inputs are the cycle's external
// inputs followed by the flip-flop outputs; after the DAG, every flip-flop latches the wire
// named for it. One HIP graph per machine holds the level sequence and the latch, and each
// cycle replays it. (CMUX memory inside the clock loop needs the address bits as TRGSW, i.e.
// circuit bootstrapping, which this parameter set does not include.)
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

void free_machine(vsp_machine* m) {
  if (!m) return;
  (void)hipSetDevice(m->ctx->device);
  (void)hipDeviceSynchronize();
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  if (m->cap) (void)hipStreamDestroy(m->cap);
  for (void* p : {(void*)m->d_next, (void*)m->d_latch})
    if (p) (void)hipFree(p);
  if (m->circ) (void)vsp_circuit_destroy(m->circ);
  delete m;
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
  if ((e = hipStreamBeginCapture(m->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return bail(hip_fail(e, "begin capture"));
  hipError_t le = circuit_launch_levels(m->circ, m->cap);
  if (le == hipSuccess && nstate) {
    uint32_t* wires = circuit_wires(m->circ);
    hipLaunchKernelGGL(k_latch_gather, dim3((unsigned)((nstate * (LWE_N + 1) + 255) / 256)), dim3(256), 0, m->cap,
                       wires, m->d_next, m->d_latch, nstate);
    le = hipGetLastError();
    if (le == hipSuccess)
      le = hipMemcpyAsync(wires + ninputs * (LWE_N + 1), m->d_latch, nstate * T0B, hipMemcpyDeviceToDevice, m->cap);
  }
  e = hipStreamEndCapture(m->cap, &m->graph);
  if (le != hipSuccess) return bail(hip_fail(le, "cycle launch during capture"));
  if (e != hipSuccess) return bail(hip_fail(e, "end capture"));
  if ((e = hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0)) != hipSuccess)
    return bail(hip_fail(e, "graph instantiate"));
  *out = m;
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
