// Levelled circuits: the per-cycle work of the paper's gate-evaluation engine (Sec. 6.2(d)),
// where every gate of a level is independent. Gates are sorted by level; each level is one
// batched launch sequence (gather inputs by wire id -> blind rotation -> key switch and
// scatter by wire id), and the whole level sequence is captured once into a HIP graph.
#include <algorithm>
#include <cstring>
#include <vector>

#include "vsp_internal.h"

using namespace vsp;

struct vsp_circuit {
  vsp_context* ctx = nullptr;
  uint64_t ngates = 0, ninputs = 0, nlevels = 0, maxw = 0;
  std::vector<uint64_t> off;         // level L occupies [off[L], off[L+1]) of the level-ordered gates
  uint8_t* d_ops = nullptr;          // level-ordered opcodes
  uint32_t* d_idx = nullptr;         // [3][ngates]: in0, in1, out wire ids (level order)
  uint32_t* d_wires = nullptr;       // [ninputs + ngates][n+1]
  uint32_t* d_abar = nullptr;        // [maxw][n+1]
  uint32_t* d_tlwe1 = nullptr;       // [maxw][N+1]
  void* d_mf = nullptr;              // matrix-core workspace, when some level is wide enough to use that form
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr size_t T0B = (LWE_N + 1) * 4;

// One level, in launch sequences of at most kMaxLaunch gates.
hipError_t launch_level(vsp_circuit* c, uint64_t L, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (uint64_t o = c->off[L]; o < c->off[L + 1] && e == hipSuccess; o += kMaxLaunch) {
    const uint64_t w = std::min<uint64_t>(kMaxLaunch, c->off[L + 1] - o);
    const uint32_t* i0 = c->d_idx + o;
    const uint32_t* i1 = c->d_idx + c->ngates + o;
    const uint32_t* io = c->d_idx + 2 * c->ngates + o;
    const uint8_t* ops = c->d_ops + o;
    e = launch_gate_prologue(c->ctx, ops, c->d_wires, c->d_wires, i0, i1, io, c->d_abar, c->d_wires, w, st);
    if (e == hipSuccess)
      e = launch_blind_rotate(c->ctx, ops, c->d_abar, c->d_tlwe1, nullptr, w, 0, st, nullptr, nullptr, nullptr, c->d_mf);
    if (e == hipSuccess) e = launch_keyswitch(c->ctx, ops, c->d_tlwe1, io, c->d_wires, w, st);
  }
  return e;
}

void free_circuit(vsp_circuit* c) {
  if (!c) return;
  (void)hipSetDevice(c->ctx->device);
  (void)hipDeviceSynchronize();
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  for (void* p : {(void*)c->d_ops, (void*)c->d_idx, (void*)c->d_wires, (void*)c->d_abar, (void*)c->d_tlwe1, c->d_mf})
    if (p) (void)hipFree(p);
  delete c;
}

}  // namespace

namespace vsp {

hipError_t circuit_launch_levels(vsp_circuit* c, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (uint64_t L = 0; L < c->nlevels && e == hipSuccess; L++) e = launch_level(c, L, st);
  return e;
}

uint32_t* circuit_wires(vsp_circuit* c) { return c->d_wires; }

}  // namespace vsp

extern "C" {

vsp_status vsp_circuit_create(vsp_context* ctx, const vsp_gate_desc* gates, uint64_t ngates, uint64_t ninputs,
                              vsp_circuit** out) {
  if (out == nullptr) return fail(VSP_E_ARG, "out is NULL");
  *out = nullptr;
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  if (ngates > 0 && gates == nullptr) return fail(VSP_E_ARG, "gates is NULL");
  if (ninputs + ngates > 0xFFFFFFFFull) return fail(VSP_E_ARG, "too many wires");
  // validate (topological order, opcodes) and levelise
  std::vector<uint32_t> lvl(ninputs + ngates, 0);
  uint64_t nlev = 0;
  for (uint64_t g = 0; g < ngates; g++) {
    const vsp_gate_desc& d = gates[g];
    const uint64_t self = ninputs + g;
    if (d.op > VSP_NOT) return fail(VSP_E_ARG, "gate " + std::to_string(g) + " has an invalid opcode");
    if (d.in0 >= self || (d.op != VSP_NOT && d.in1 >= self))
      return fail(VSP_E_ARG, "gate " + std::to_string(g) + " reads a wire that is not computed before it");
    uint32_t L = lvl[d.in0];
    if (d.op != VSP_NOT) L = std::max(L, lvl[d.in1]);
    lvl[self] = L + 1;
    nlev = std::max<uint64_t>(nlev, L + 1);
  }
  auto* c = new vsp_circuit();
  c->ctx = ctx;
  c->ngates = ngates;
  c->ninputs = ninputs;
  c->nlevels = nlev;
  c->off.assign(nlev + 1, 0);
  for (uint64_t g = 0; g < ngates; g++) c->off[lvl[ninputs + g]]++;  // counts at index level (1-based)
  // prefix sums: level L (1-based) -> slot L-1
  std::vector<uint64_t> start(nlev + 1, 0);
  for (uint64_t L = 1; L <= nlev; L++) start[L] = start[L - 1] + c->off[L];
  for (uint64_t L = 0; L <= nlev; L++) c->off[L] = start[L];
  for (uint64_t L = 0; L < nlev; L++) c->maxw = std::max(c->maxw, c->off[L + 1] - c->off[L]);
  std::vector<uint64_t> pos(start.begin(), start.end() - 1);
  std::vector<uint8_t> hops(ngates);
  std::vector<uint32_t> hidx(3 * ngates);
  for (uint64_t g = 0; g < ngates; g++) {
    const uint64_t p = pos[lvl[ninputs + g] - 1]++;
    hops[p] = (uint8_t)gates[g].op;
    hidx[p] = gates[g].in0;
    hidx[ngates + p] = gates[g].op == VSP_NOT ? gates[g].in0 : gates[g].in1;
    hidx[2 * ngates + p] = (uint32_t)(ninputs + g);
  }
  auto bail = [&](vsp_status s) {
    free_circuit(c);
    return s;
  };
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return bail(hip_fail(e, "hipSetDevice"));
  const uint64_t wmax = std::max<uint64_t>(std::min<uint64_t>(c->maxw, kMaxLaunch), 1);
  if ((e = hipMalloc(&c->d_ops, std::max<uint64_t>(ngates, 1))) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
  if ((e = hipMalloc(&c->d_idx, std::max<uint64_t>(3 * ngates, 1) * 4)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
  if ((e = hipMalloc(&c->d_wires, std::max<uint64_t>(ninputs + ngates, 1) * T0B)) != hipSuccess)
    return bail(hip_fail(e, "hipMalloc(wires)"));
  if ((e = hipMalloc(&c->d_abar, wmax * T0B)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
  if ((e = hipMalloc(&c->d_tlwe1, wmax * (RING_N + 1) * 4)) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
  bool matrix = false;  // the launch choice is fixed when the level sequence is captured below
  for (uint64_t L = 0; L < nlev && ctx->mf_key; L++)
    matrix |= br_matrix_form(ctx->tune.br_waves(std::min<uint64_t>(kMaxLaunch, c->off[L + 1] - c->off[L])));
  if (matrix && (e = hipMalloc(&c->d_mf, mf_work_bytes(wmax, true))) != hipSuccess) return bail(hip_fail(e, "hipMalloc"));
  if (ngates) {
    if ((e = hipMemcpy(c->d_ops, hops.data(), ngates, hipMemcpyHostToDevice)) != hipSuccess) return bail(hip_fail(e, "upload"));
    if ((e = hipMemcpy(c->d_idx, hidx.data(), 3 * ngates * 4, hipMemcpyHostToDevice)) != hipSuccess)
      return bail(hip_fail(e, "upload"));
  }
  // capture the level sequence into a graph
  if ((e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking)) != hipSuccess) return bail(hip_fail(e, "stream"));
  if ((e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return bail(hip_fail(e, "begin capture"));
  const hipError_t le = circuit_launch_levels(c, c->cap);
  e = hipStreamEndCapture(c->cap, &c->graph);
  if (le != hipSuccess) return bail(hip_fail(le, "level launch during capture"));
  if (e != hipSuccess) return bail(hip_fail(e, "end capture"));
  if ((e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0)) != hipSuccess)
    return bail(hip_fail(e, "graph instantiate"));
  *out = c;
  return VSP_OK;
}

static vsp_status circuit_io_check(vsp_circuit* c, const uint32_t* d_inputs, uint32_t* d_wires) {
  if (c == nullptr) return fail(VSP_E_ARG, "circuit is NULL");
  vsp_status s;
  const size_t ib = c->ninputs * T0B, wb = (c->ninputs + c->ngates) * T0B;
  if (ib && (s = check_device_range(c->ctx, d_inputs, ib, "d_inputs"))) return s;
  if (wb && (s = check_device_range(c->ctx, d_wires, wb, "d_wires"))) return s;
  if (ib && wb && d_inputs != d_wires && (s = check_no_overlap(d_wires, wb, d_inputs, ib, "d_wires and d_inputs")))
    return s;
  return VSP_OK;
}

vsp_status vsp_circuit_run(vsp_circuit* c, const uint32_t* d_inputs, uint32_t* d_wires, void* stream) {
  vsp_status s = circuit_io_check(c, d_inputs, d_wires);
  if (s) return s;
  VSP_HIP(hipSetDevice(c->ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (c->ninputs) VSP_HIP(hipMemcpyAsync(c->d_wires, d_inputs, c->ninputs * T0B, hipMemcpyDeviceToDevice, st));
  if (c->nlevels) VSP_HIP(hipGraphLaunch(c->exec, st));
  const size_t wb = (c->ninputs + c->ngates) * T0B;
  if (wb) VSP_HIP(hipMemcpyAsync(d_wires, c->d_wires, wb, hipMemcpyDeviceToDevice, st));
  return VSP_OK;
}

vsp_status vsp_circuit_run_timed(vsp_circuit* c, const uint32_t* d_inputs, uint32_t* d_wires, void* stream,
                                 float* h_level_ms) {
  vsp_status s = circuit_io_check(c, d_inputs, d_wires);
  if (s) return s;
  if (c->nlevels && h_level_ms == nullptr) return fail(VSP_E_ARG, "h_level_ms is NULL");
  VSP_HIP(hipSetDevice(c->ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (c->ninputs) VSP_HIP(hipMemcpyAsync(c->d_wires, d_inputs, c->ninputs * T0B, hipMemcpyDeviceToDevice, st));
  std::vector<hipEvent_t> ev(c->nlevels + 1);
  for (auto& x : ev) VSP_HIP(hipEventCreate(&x));
  VSP_HIP(hipEventRecord(ev[0], st));
  for (uint64_t L = 0; L < c->nlevels; L++) {
    hipError_t e = launch_level(c, L, st);
    if (e != hipSuccess) return hip_fail(e, "level launch");
    VSP_HIP(hipEventRecord(ev[L + 1], st));
  }
  VSP_HIP(hipEventSynchronize(ev[c->nlevels]));
  for (uint64_t L = 0; L < c->nlevels; L++) VSP_HIP(hipEventElapsedTime(&h_level_ms[L], ev[L], ev[L + 1]));
  for (auto& x : ev) (void)hipEventDestroy(x);
  const size_t wb = (c->ninputs + c->ngates) * T0B;
  if (wb) VSP_HIP(hipMemcpyAsync(d_wires, c->d_wires, wb, hipMemcpyDeviceToDevice, st));
  VSP_HIP(hipStreamSynchronize(st));
  return VSP_OK;
}

vsp_status vsp_circuit_info(const vsp_circuit* c, uint64_t* nlevels, uint64_t* max_width) {
  if (c == nullptr || nlevels == nullptr || max_width == nullptr) return fail(VSP_E_ARG, "NULL argument");
  *nlevels = c->nlevels;
  *max_width = c->maxw;
  return VSP_OK;
}

vsp_status vsp_circuit_destroy(vsp_circuit* c) {
  free_circuit(c);
  return VSP_OK;
}

}  // extern "C"
