// C ABI of libvsp: status codes, the context, batched / per-gate homomorphic gates,
// TRLWE-output bootstrapping and the test entry points. CMUX memory, circuits and the
// server have their own files.
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "vsp_internal.h"

namespace vsp {

static thread_local std::string g_last_error;

vsp_status fail(vsp_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

vsp_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? VSP_E_NOMEM : VSP_E_HIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

vsp_status check_device_range(const vsp_context* ctx, const void* p, size_t bytes, const char* name) {
  if (p == nullptr) return fail(VSP_E_ARG, std::string(name) + " is NULL");
  if (reinterpret_cast<uintptr_t>(p) & 3u) return fail(VSP_E_ARG, std::string(name) + " is not 4-byte aligned");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(VSP_E_ARG, std::string(name) + " is not device memory");
  }
  if (attr.type != hipMemoryTypeDevice && !attr.isManaged)
    return fail(VSP_E_ARG, std::string(name) + " is not device memory");
  if (attr.device != ctx->device)
    return fail(VSP_E_ARG, std::string(name) + " lives on another device");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(VSP_E_ARG, std::string(name) + ": cannot query its allocation");
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(p);
  if (q < b || (size_t)(q - b) + bytes > size)
    return fail(VSP_E_ARG, std::string(name) + " is smaller than the " + std::to_string(bytes) + " bytes needed");
  return VSP_OK;
}

vsp_status check_no_overlap(const void* a, size_t abytes, const void* b, size_t bbytes, const char* what) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  if (x < y + bbytes && y < x + abytes) return fail(VSP_E_ARG, std::string(what) + " overlap");
  return VSP_OK;
}

vsp_status scratch_reserve(vsp_context* ctx, Scratch& s, size_t bytes) {
  if (s.bytes >= bytes) return VSP_OK;
  if (s.ptr) {
    VSP_HIP(hipDeviceSynchronize());
    VSP_HIP(hipFree(s.ptr));
    s.ptr = nullptr;
    s.bytes = 0;
  }
  size_t want = bytes + bytes / 4;
  VSP_HIP(hipMalloc(&s.ptr, want));
  s.bytes = want;
  return VSP_OK;
}

ProfScope::ProfScope(const vsp_context* c, int w, hipStream_t s, uint32_t launches) : ctx(c), which(w), st(s) {
  if (ctx == nullptr || !ctx->prof.on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return;
  }
  if (ctx->prof.seen[which]++ % (uint64_t)ctx->prof.period != 0) return;
  hipEvent_t e0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    e1 = nullptr;
    return;
  }
  (void)hipEventRecord(e0, st);
  ctx->prof.ev[which].push_back({e0, e1, launches});
}

ProfScope::~ProfScope() {
  if (e1) (void)hipEventRecord(e1, st);
}

static void profile_clear(vsp_context* ctx) {
  for (auto& v : ctx->prof.ev) {
    for (auto& p : v) {
      (void)hipEventDestroy(p.e0);
      (void)hipEventDestroy(p.e1);
    }
    v.clear();
  }
}

// ------------------------------------------------------------------ host twiddle tables
static u64 h_mulmod(u64 a, u64 b) { return (u64)(((unsigned __int128)a * b) % GL_P); }
static u64 h_powmod(u64 b, u64 e) {
  u64 r = 1;
  b %= GL_P;
  while (e) {
    if (e & 1) r = h_mulmod(r, b);
    b = h_mulmod(b, b);
    e >>= 1;
  }
  return r;
}

// psi: a primitive 2048th root of unity with psi^32 = 8 (so psi_u^32 = 8^{2u+1} = zeta_u).
// 7 generates the multiplicative group mod p.
static bool make_tables(std::vector<u64>& tw) {
  const u64 psi0 = h_powmod(7, (GL_P - 1) / 2048);
  if (h_powmod(psi0, 1024) != GL_P - 1) return false;
  const u64 w = h_powmod(psi0, 32);
  int m = -1;
  for (int c = 0; c < 64; c++)
    if (h_powmod(w, c) == 8) { m = c; break; }
  if (m < 0) return false;
  const u64 psi = h_powmod(psi0, m);
  if (h_powmod(psi, 32) != 8 || h_powmod(psi, 1024) != GL_P - 1) return false;
  tw.assign(2048, 0);
  for (int j = 0; j < 32; j++)
    for (int u = 0; u < 32; u++) {
      const int e = ((2 * u + 1) * j) % 2048;
      tw[j * 32 + u] = h_powmod(psi, e);
      tw[1024 + j * 32 + u] = h_powmod(psi, (2048 - e) % 2048);
    }
  return true;
}

vsp_status upload_keys(const vsp_context* ctx, const uint32_t* bk_host, const uint32_t* ksk_host, uint64_t** bkn,
                       uint32_t** ksk, int8_t** mf_key, int8_t** ks_mf) {
  *bkn = nullptr;
  *ksk = nullptr;
  if (mf_key) *mf_key = nullptr;
  if (ks_mf) *ks_mf = nullptr;
  const size_t bk_words = (size_t)LWE_N * 2 * GADGET_L * 2 * RING_N;
  const size_t ksk_rows = (size_t)RING_N * KS_T * 4;
  uint64_t* b = nullptr;
  uint32_t* k = nullptr;
  uint32_t* tmp = nullptr;
  int8_t* E = nullptr;
  int8_t* KM = nullptr;
  auto undo = [&](vsp_status st) {
    for (void* p : {(void*)b, (void*)k, (void*)tmp, (void*)E, (void*)KM})
      if (p) (void)hipFree(p);
    return st;
  };
  hipError_t e;
  if ((e = hipMalloc(&b, (size_t)LWE_N * TRGSW_NTT_U64 * 8)) != hipSuccess) return undo(hip_fail(e, "hipMalloc(bk)"));
  if ((e = hipMalloc(&k, ksk_rows * (LWE_N + 1) * 4)) != hipSuccess) return undo(hip_fail(e, "hipMalloc(ksk)"));
  // Bootstrapping key: torus -> NTT domain on the device.
  if ((e = hipMalloc(&tmp, bk_words * 4)) != hipSuccess) return undo(hip_fail(e, "hipMalloc(bk staging)"));
  e = hipMemcpy(tmp, bk_host, bk_words * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_trgsw_to_ntt(ctx, tmp, b, LWE_N, nullptr);
  if (e == hipSuccess && mf_key) {
    e = hipMalloc(&E, mf_key_bytes());
    if (e == hipSuccess) e = launch_mf_key(tmp, E, nullptr);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return undo(hip_fail(e, "bootstrapping-key conversion"));
  (void)hipFree(tmp);
  tmp = nullptr;
  // Key-switching key, with a zero row in front of the three digit rows of every (j, p).
  std::vector<uint32_t> k4(ksk_rows * (LWE_N + 1), 0u);
  for (size_t jp = 0; jp < (size_t)RING_N * KS_T; jp++)
    for (int v = 1; v < 4; v++)
      std::memcpy(&k4[(jp * 4 + v) * (LWE_N + 1)], &ksk_host[(jp * 3 + (v - 1)) * (LWE_N + 1)], (LWE_N + 1) * 4);
  if ((e = hipMemcpy(k, k4.data(), k4.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return undo(hip_fail(e, "upload ksk"));
  if (ks_mf) {
    if ((e = hipMalloc(&KM, ks_mf_key_bytes())) != hipSuccess) return undo(hip_fail(e, "hipMalloc(ks bytes)"));
    if ((e = launch_ks_mfkey(k, KM, nullptr)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess)
      return undo(hip_fail(e, "key-switching key conversion"));
  }
  *bkn = b;
  *ksk = k;
  if (mf_key) *mf_key = E;
  if (ks_mf) *ks_mf = KM;
  return VSP_OK;
}

static vsp_status check_ctx(const vsp_context* ctx) {
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  return VSP_OK;
}

}  // namespace vsp

using namespace vsp;

extern "C" {

const char* vsp_status_str(vsp_status s) {
  switch (s) {
    case VSP_OK: return "ok";
    case VSP_E_ARG: return "invalid argument";
    case VSP_E_PARAMS: return "parameter set differs from the compiled one";
    case VSP_E_NOMEM: return "device allocation failed";
    case VSP_E_HIP: return "HIP runtime or kernel failure";
    case VSP_E_STATE: return "object in the wrong state";
    case VSP_E_CAPACITY: return "request exceeds the memory budget";
    default: return "unknown status";
  }
}

const char* vsp_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------ allocation-free gates
// Fixed device scratch of vsp_gates_noalloc: the modulus-switched inputs ([kStaticGates][n+1])
// and the extracted TLWE rows ([kStaticGates][N+1]) of one call. Each device holds its own
// copy at its own address, resolved once per device (with that device current) when the first
// context on it is created; host code uses only that address, never the array's name.
constexpr uint64_t kStaticGates = 2048;
constexpr size_t kStaticAbarBytes = (size_t)kStaticGates * TLWE0 * 4;
constexpr size_t kStaticBytes = kStaticAbarBytes + (size_t)kStaticGates * TLWE1 * 4;
static_assert(kStaticAbarBytes % 256 == 0, "the extracted rows start 256-byte aligned");
static __device__ __align__(256) uint8_t scratch[kStaticBytes];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;  // indexed by device; null until resolved

static vsp_status resolve_static_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((size_t)device < g_scratch_ptr.size() && g_scratch_ptr[device] != nullptr) return VSP_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (p == nullptr) return fail(VSP_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
  if ((size_t)device >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)device + 1, nullptr);
  g_scratch_ptr[device] = p;
  return VSP_OK;
}

static void* static_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (size_t)device < g_scratch_ptr.size() ? g_scratch_ptr[device] : nullptr;
}

vsp_status vsp_context_create(const vsp_params* params, const uint32_t* bk_host, const uint32_t* ksk_host, int device,
                              vsp_context** out) {
  if (out == nullptr) return fail(VSP_E_ARG, "out is NULL");
  *out = nullptr;
  if (params == nullptr || bk_host == nullptr || ksk_host == nullptr)
    return fail(VSP_E_ARG, "params, bk_host and ksk_host must not be NULL");
  if (params->n != LWE_N || params->N != RING_N || params->k != 1 || params->l != GADGET_L ||
      params->bg_bits != BG_BIT || params->ks_t != KS_T || params->ks_basebit != KS_BASEBIT)
    return fail(VSP_E_PARAMS, "the library supports n=630 N=1024 k=1 l=3 bg_bits=6 ks_t=8 ks_basebit=2 only");
  int ndev = 0;
  VSP_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(VSP_E_ARG, "no such device");
  VSP_HIP(hipSetDevice(device));
  VSP_HIP(init_kernel_attributes());
  VSP_HIP(init_memory_kernel_attributes());
  VSP_HIP(init_mf_kernel_attributes());
  if (vsp_status st = resolve_static_scratch(device)) return st;
  std::vector<u64> tw;
  if (!make_tables(tw)) return fail(VSP_E_HIP, "twiddle table construction failed");

  auto* ctx = new vsp_context();
  ctx->device = device;
  auto cleanup = [&](vsp_status s) {
    vsp_context_destroy(ctx);
    return s;
  };
  {
    hipError_t e = blind_rotate_capacity(device, ctx->tune.br_cap);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return cleanup(hip_fail(e, "occupancy query"));
  }
  hipError_t e;
  if ((e = hipMalloc(&ctx->tw, tw.size() * 8)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc(tw)"));
  if ((e = hipMalloc(&ctx->dev_err, 256)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc(err)"));
  if ((e = hipMemcpy(ctx->tw, tw.data(), tw.size() * 8, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(e, "upload twiddles"));
  if ((e = hipMemset(ctx->dev_err, 0, 256)) != hipSuccess) return cleanup(hip_fail(e, "clear flags"));
  if (vsp_status st = upload_keys(ctx, bk_host, ksk_host, &ctx->bkn, &ctx->ksk, &ctx->mf_key, &ctx->ks_mf))
    return cleanup(st);
  *out = ctx;
  return VSP_OK;
}

vsp_status vsp_context_destroy(vsp_context* ctx) {
  if (ctx == nullptr) return VSP_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  profile_clear(ctx);
  for (void* p : {(void*)ctx->bkn, (void*)ctx->ksk, (void*)ctx->mf_key, (void*)ctx->ks_mf, (void*)ctx->tw,
                  (void*)ctx->dev_err,
                  ctx->abar.ptr, ctx->tlwe1.ptr, ctx->ntt_sel.ptr, ctx->mem_a.ptr, ctx->mem_b.ptr, ctx->mem_c.ptr,
                  ctx->mem_d.ptr, ctx->mf_work.ptr})
    if (p) (void)hipFree(p);
  delete ctx;
  return VSP_OK;
}

vsp_status vsp_context_sync(vsp_context* ctx) {
  vsp_status s = check_ctx(ctx);
  if (s) return s;
  VSP_HIP(hipSetDevice(ctx->device));
  VSP_HIP(hipDeviceSynchronize());
  int flags = 0;
  VSP_HIP(hipMemcpy(&flags, ctx->dev_err, sizeof(int), hipMemcpyDeviceToHost));
  if (flags) {
    VSP_HIP(hipMemset(ctx->dev_err, 0, sizeof(int)));
    if (flags & DEVERR_BAD_OP) return fail(VSP_E_ARG, "a gate had an invalid opcode (its output was zeroed)");
  }
  return VSP_OK;
}

// Argument checks shared by the gate entry points.
static vsp_status check_gate_args(vsp_context* ctx, const uint8_t* d_ops, const uint32_t* d_in0, const uint32_t* d_in1,
                                  uint32_t* d_out, uint64_t B, int mode, bool trlwe_out) {
  vsp_status s;
  if (mode != VSP_BATCHED && mode != VSP_PER_GATE) return fail(VSP_E_ARG, "mode must be VSP_BATCHED or VSP_PER_GATE");
  if (B > (1ull << 31)) return fail(VSP_E_ARG, "B too large");
  const size_t tl = (size_t)B * (LWE_N + 1) * 4;
  const size_t ob = trlwe_out ? (size_t)B * 2 * RING_N * 4 : tl;
  if ((s = check_device_range(ctx, d_ops, B, "d_ops"))) return s;
  if ((s = check_device_range(ctx, d_in0, tl, "d_in0"))) return s;
  if ((s = check_device_range(ctx, d_in1, tl, "d_in1"))) return s;
  if ((s = check_device_range(ctx, d_out, ob, "d_out"))) return s;
  if ((s = check_no_overlap(d_out, ob, d_in0, tl, "d_out and d_in0"))) return s;
  if ((s = check_no_overlap(d_out, ob, d_in1, tl, "d_out and d_in1"))) return s;
  if ((s = check_no_overlap(d_out, ob, d_ops, B, "d_out and d_ops"))) return s;
  return VSP_OK;
}

// Enqueues prologue -> blind rotation -> key switch (or the TRLWE output) for B gates in
// chunks of `chunk`, with the modulus-switched inputs in abar (chunk rows), the extracted rows
// in t1 (chunk rows) and the matrix-core workspace mfw (NULL: the NTT forms).
static vsp_status gates_enqueue(vsp_context* ctx, const uint8_t* d_ops, const uint32_t* d_in0, const uint32_t* d_in1,
                                uint32_t* d_out, uint64_t B, uint64_t chunk, bool trlwe_out, uint32_t* abar,
                                uint32_t* t1, void* mfw, hipStream_t st, bool prof) {
  const vsp_context* pc = prof ? ctx : nullptr;
  for (uint64_t g0 = 0; g0 < B; g0 += chunk) {
    const uint64_t nb = (B - g0 < chunk) ? B - g0 : chunk;
    const uint8_t* ops = d_ops + g0;
    const uint32_t* i0 = d_in0 + g0 * (LWE_N + 1);
    const uint32_t* i1 = d_in1 + g0 * (LWE_N + 1);
    hipError_t e;
    if (trlwe_out) {
      uint32_t* o = d_out + g0 * 2 * RING_N;
      // NOT / invalid opcodes are reported through the device flag; their TRLWE stays untouched.
      {
        ProfScope ps(pc, 2, st);
        e = launch_gate_prologue(ctx, ops, i0, i1, nullptr, nullptr, nullptr, abar, nullptr, nb, st, false);
      }
      if (e != hipSuccess) return hip_fail(e, "gate prologue");
      {
        ProfScope ps(pc, 0, st);
        e = launch_blind_rotate(ctx, ops, abar, nullptr, o, nb, 0, st, nullptr, nullptr, nullptr, mfw, prof);
      }
      if (e != hipSuccess) return hip_fail(e, "blind rotation");
    } else {
      uint32_t* o = d_out + g0 * (LWE_N + 1);
      {
        ProfScope ps(pc, 2, st);
        e = launch_gate_prologue(ctx, ops, i0, i1, nullptr, nullptr, nullptr, abar, o, nb, st);
      }
      if (e != hipSuccess) return hip_fail(e, "gate prologue");
      {
        ProfScope ps(pc, 0, st);
        e = launch_blind_rotate(ctx, ops, abar, t1, nullptr, nb, 0, st, nullptr, nullptr, nullptr, mfw, prof);
      }
      if (e != hipSuccess) return hip_fail(e, "blind rotation");
      {
        ProfScope ps(pc, 1, st);
        e = launch_keyswitch(ctx, ops, t1, nullptr, o, nb, st);
      }
      if (e != hipSuccess) return hip_fail(e, "key switch");
    }
  }
  return VSP_OK;
}

static vsp_status gates_impl(vsp_context* ctx, const uint8_t* d_ops, const uint32_t* d_in0, const uint32_t* d_in1,
                             uint32_t* d_out, uint64_t B, int mode, void* stream, bool trlwe_out) {
  vsp_status s = check_ctx(ctx);
  if (s) return s;
  if (mode != VSP_BATCHED && mode != VSP_PER_GATE) return fail(VSP_E_ARG, "mode must be VSP_BATCHED or VSP_PER_GATE");
  if (B == 0) return VSP_OK;
  VSP_HIP(hipSetDevice(ctx->device));
  if ((s = check_gate_args(ctx, d_ops, d_in0, d_in1, d_out, B, mode, trlwe_out))) return s;
  const uint64_t chunk = (mode == VSP_BATCHED) ? std::min<uint64_t>(B, kMaxLaunch) : 1;
  if ((s = scratch_reserve(ctx, ctx->abar, chunk * (LWE_N + 1) * 4))) return s;
  if (!trlwe_out && (s = scratch_reserve(ctx, ctx->tlwe1, chunk * (RING_N + 1) * 4))) return s;
  const bool matrix =
      br_matrix_form(ctx->tune.br_waves(chunk)) || (B > chunk && br_matrix_form(ctx->tune.br_waves(B % chunk)));
  if (matrix && (s = scratch_reserve(ctx, ctx->mf_work, mf_work_bytes(chunk, !trlwe_out)))) return s;
  void* mfw = matrix ? ctx->mf_work.ptr : nullptr;
  return gates_enqueue(ctx, d_ops, d_in0, d_in1, d_out, B, chunk, trlwe_out, static_cast<uint32_t*>(ctx->abar.ptr),
                       static_cast<uint32_t*>(ctx->tlwe1.ptr), mfw, static_cast<hipStream_t>(stream), true);
}


vsp_status vsp_gates(vsp_context* ctx, const uint8_t* d_ops, const uint32_t* d_in0, const uint32_t* d_in1,
                     uint32_t* d_out, uint64_t B, int mode, void* stream) {
  return gates_impl(ctx, d_ops, d_in0, d_in1, d_out, B, mode, stream, false);
}

vsp_status vsp_gates_noalloc(vsp_context* ctx, const uint8_t* d_ops, const uint32_t* d_in0, const uint32_t* d_in1,
                             uint32_t* d_out, uint64_t B, int mode, void* stream) {
  vsp_status s = check_ctx(ctx);
  if (s) return s;
  if (mode != VSP_BATCHED && mode != VSP_PER_GATE) return fail(VSP_E_ARG, "mode must be VSP_BATCHED or VSP_PER_GATE");
  if (B > kStaticGates)
    return fail(VSP_E_ARG, "vsp_gates_noalloc takes at most " + std::to_string(kStaticGates) + " gates per call (got " +
                               std::to_string(B) + ")");
  if (B == 0) return VSP_OK;
  VSP_HIP(hipSetDevice(ctx->device));
  if ((s = check_gate_args(ctx, d_ops, d_in0, d_in1, d_out, B, mode, false))) return s;
  uint8_t* base = static_cast<uint8_t*>(static_scratch(ctx->device));
  if (base == nullptr) return fail(VSP_E_STATE, "the static scratch of this device was not resolved");
  const uint64_t chunk = (mode == VSP_BATCHED) ? B : 1;
  // no matrix-core workspace: the NTT forms of the blind rotation (the key switch needs none)
  return gates_enqueue(ctx, d_ops, d_in0, d_in1, d_out, B, chunk, false, reinterpret_cast<uint32_t*>(base),
                       reinterpret_cast<uint32_t*>(base + kStaticAbarBytes), nullptr,
                       static_cast<hipStream_t>(stream), false);
}

vsp_status vsp_bootstrap_trlwe(vsp_context* ctx, const uint8_t* d_ops, const uint32_t* d_in0, const uint32_t* d_in1,
                               uint32_t* d_out, uint64_t B, void* stream) {
  return gates_impl(ctx, d_ops, d_in0, d_in1, d_out, B, VSP_BATCHED, stream, true);
}

vsp_status vsp_gates_key_copies(vsp_context* ctx, const uint8_t* d_ops, const uint32_t* d_in0, const uint32_t* d_in1,
                                uint32_t* d_out, uint64_t B, int waves, uint32_t copies, void* stream,
                                double* br_ms) {
  vsp_status s = check_ctx(ctx);
  if (s) return s;
  if (waves != 3 && waves != 4 && waves != 8) return fail(VSP_E_ARG, "waves must be 3, 4 or 8 (an NTT form)");
  if (copies == 0 || copies > 65536) return fail(VSP_E_ARG, "copies must be in [1, 65536]");
  if (br_ms == nullptr) return fail(VSP_E_ARG, "br_ms must be non-NULL");
  if (B > kMaxLaunch) return fail(VSP_E_ARG, "B above one launch (" + std::to_string(kMaxLaunch) + " gates)");
  *br_ms = 0;
  if (B == 0) return VSP_OK;
  VSP_HIP(hipSetDevice(ctx->device));
  if ((s = check_gate_args(ctx, d_ops, d_in0, d_in1, d_out, B, VSP_BATCHED, false))) return s;
  const size_t key_bytes = (size_t)LWE_N * TRGSW_NTT_U64 * 8;
  const size_t copy_bytes = copies > 1 ? (size_t)copies * key_bytes : 0;
  size_t free_b = 0, total_b = 0;
  VSP_HIP(hipMemGetInfo(&free_b, &total_b));
  if (copy_bytes + (1ull << 30) > free_b)
    return fail(VSP_E_NOMEM, std::to_string(copies) + " key copies need " + std::to_string(copy_bytes >> 20) +
                                 " MiB; " + std::to_string(free_b >> 20) + " MiB free on the device");
  if ((s = scratch_reserve(ctx, ctx->abar, B * (LWE_N + 1) * 4))) return s;
  if ((s = scratch_reserve(ctx, ctx->tlwe1, B * (RING_N + 1) * 4))) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint64_t* keys = nullptr;
  const uint64_t** d_tab = nullptr;
  uint16_t* d_kid = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto undo = [&](vsp_status r) {
    if (st) (void)hipStreamSynchronize(st);
    else (void)hipDeviceSynchronize();
    for (void* p : {(void*)keys, (void*)d_tab, (void*)d_kid})
      if (p) (void)hipFree(p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return r;
  };
  hipError_t e;
  std::vector<const uint64_t*> tab(copies, ctx->bkn);
  if (copies > 1) {
    if ((e = hipMalloc(&keys, copy_bytes)) != hipSuccess) return undo(hip_fail(e, "hipMalloc(key copies)"));
    for (uint32_t c = 0; c < copies; c++) {
      tab[c] = keys + (size_t)c * LWE_N * TRGSW_NTT_U64;
      if ((e = hipMemcpyAsync(keys + (size_t)c * LWE_N * TRGSW_NTT_U64, ctx->bkn, key_bytes, hipMemcpyDeviceToDevice,
                              st)) != hipSuccess)
        return undo(hip_fail(e, "key copy"));
    }
  }
  std::vector<uint16_t> kid(B);
  for (uint64_t g = 0; g < B; g++) kid[g] = (uint16_t)(g % copies);
  if ((e = hipMalloc(&d_tab, copies * sizeof(void*))) != hipSuccess) return undo(hip_fail(e, "hipMalloc(key table)"));
  if ((e = hipMalloc(&d_kid, B * sizeof(uint16_t))) != hipSuccess) return undo(hip_fail(e, "hipMalloc(key index)"));
  if ((e = hipMemcpyAsync(d_tab, tab.data(), copies * sizeof(void*), hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(d_kid, kid.data(), B * sizeof(uint16_t), hipMemcpyHostToDevice, st)) != hipSuccess)
    return undo(hip_fail(e, "key table upload"));
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    return undo(hip_fail(e, "hipEventCreate"));
  uint32_t* abar = static_cast<uint32_t*>(ctx->abar.ptr);
  uint32_t* t1 = static_cast<uint32_t*>(ctx->tlwe1.ptr);
  if ((e = launch_gate_prologue(ctx, d_ops, d_in0, d_in1, nullptr, nullptr, nullptr, abar, d_out, B, st)) !=
      hipSuccess)
    return undo(hip_fail(e, "gate prologue"));
  (void)hipEventRecord(e0, st);
  e = launch_blind_rotate(ctx, d_ops, abar, t1, nullptr, B, waves, st, nullptr, d_tab, d_kid);
  (void)hipEventRecord(e1, st);
  if (e != hipSuccess) return undo(hip_fail(e, "blind rotation"));
  if ((e = launch_keyswitch(ctx, d_ops, t1, nullptr, d_out, B, st)) != hipSuccess) return undo(hip_fail(e, "key switch"));
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return undo(hip_fail(e, "hipStreamSynchronize"));
  float ms = 0;
  if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return undo(hip_fail(e, "hipEventElapsedTime"));
  *br_ms = ms;
  return undo(VSP_OK);
}

vsp_status vsp_keyset_create(vsp_context* ctx, const uint32_t* bk_host, const uint32_t* ksk_host, vsp_keyset** out) {
  if (out == nullptr) return fail(VSP_E_ARG, "out is NULL");
  *out = nullptr;
  vsp_status s = check_ctx(ctx);
  if (s) return s;
  if (bk_host == nullptr || ksk_host == nullptr) return fail(VSP_E_ARG, "bk_host and ksk_host must not be NULL");
  VSP_HIP(hipSetDevice(ctx->device));
  auto* k = new vsp_keyset();
  k->ctx = ctx;
  if ((s = upload_keys(ctx, bk_host, ksk_host, &k->bkn, &k->ksk, &k->mf_key, &k->ks_mf))) {
    delete k;
    return s;
  }
  *out = k;
  return VSP_OK;
}

vsp_status vsp_keyset_destroy(vsp_keyset* k) {
  if (k == nullptr) return VSP_OK;
  (void)hipSetDevice(k->ctx->device);
  (void)hipDeviceSynchronize();
  for (void* p : {(void*)k->bkn, (void*)k->ksk, (void*)k->mf_key, (void*)k->ks_mf})
    if (p) (void)hipFree(p);
  delete k;
  return VSP_OK;
}

vsp_status vsp_mux(vsp_context* ctx, const uint32_t* d_sel, const uint32_t* d_in1, const uint32_t* d_in0,
                   uint32_t* d_out, uint64_t B, void* stream) {
  vsp_status s = check_ctx(ctx);
  if (s) return s;
  if (B == 0) return VSP_OK;
  if (B > (1ull << 30)) return fail(VSP_E_ARG, "B too large");
  VSP_HIP(hipSetDevice(ctx->device));
  const size_t tl = (size_t)B * (LWE_N + 1) * 4;
  if ((s = check_device_range(ctx, d_sel, tl, "d_sel"))) return s;
  if ((s = check_device_range(ctx, d_in1, tl, "d_in1"))) return s;
  if ((s = check_device_range(ctx, d_in0, tl, "d_in0"))) return s;
  if ((s = check_device_range(ctx, d_out, tl, "d_out"))) return s;
  if ((s = check_no_overlap(d_out, tl, d_sel, tl, "d_out and d_sel"))) return s;
  if ((s = check_no_overlap(d_out, tl, d_in1, tl, "d_out and d_in1"))) return s;
  if ((s = check_no_overlap(d_out, tl, d_in0, tl, "d_out and d_in0"))) return s;
  const uint64_t chunk = std::min<uint64_t>(B, kMaxLaunch / 2);
  if ((s = scratch_reserve(ctx, ctx->abar, 2 * chunk * (LWE_N + 1) * 4))) return s;
  if ((s = scratch_reserve(ctx, ctx->tlwe1, 2 * chunk * (RING_N + 1) * 4))) return s;
  // the 2B bootstraps take the matrix-core forms where the tuning picks them (one workspace)
  const bool matrix = br_matrix_form(ctx->tune.br_waves(2 * chunk)) ||
                      (B > chunk && br_matrix_form(ctx->tune.br_waves(2 * (B % chunk))));
  if (matrix && (s = scratch_reserve(ctx, ctx->mf_work, mf_work_bytes(2 * chunk, true)))) return s;
  void* mfw = matrix ? ctx->mf_work.ptr : nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t* abar = static_cast<uint32_t*>(ctx->abar.ptr);
  uint32_t* t1 = static_cast<uint32_t*>(ctx->tlwe1.ptr);
  for (uint64_t g0 = 0; g0 < B; g0 += chunk) {
    const uint64_t nb = std::min<uint64_t>(chunk, B - g0);
    const size_t o = g0 * (LWE_N + 1);
    hipError_t e;
    {
      ProfScope ps(ctx, 2, st);
      e = launch_mux_prologue(d_sel + o, d_in1 + o, d_in0 + o, abar, nb, st);
    }
    if (e != hipSuccess) return hip_fail(e, "mux prologue");
    {
      ProfScope ps(ctx, 0, st);
      e = launch_blind_rotate(ctx, nullptr, abar, t1, nullptr, 2 * nb, 0, st, nullptr, nullptr, nullptr, mfw);
    }
    if (e != hipSuccess) return hip_fail(e, "blind rotation");
    if ((e = launch_mux_combine(t1, nb, st)) != hipSuccess) return hip_fail(e, "mux combine");
    {
      ProfScope ps(ctx, 1, st);
      e = launch_keyswitch(ctx, nullptr, t1, nullptr, d_out + o, nb, st);
    }
    if (e != hipSuccess) return hip_fail(e, "key switch");
  }
  return VSP_OK;
}

vsp_status vsp_profile_enable(vsp_context* ctx, int on) {
  vsp_status s = check_ctx(ctx);
  if (s) return s;
  VSP_HIP(hipSetDevice(ctx->device));
  if (on < 0) return fail(VSP_E_ARG, "on must be 0 (off), 1 (every launch) or a sampling period");
  VSP_HIP(hipDeviceSynchronize());
  profile_clear(ctx);
  ctx->prof.on = on != 0;
  ctx->prof.period = on > 1 ? on : 1;
  for (auto& n : ctx->prof.seen) n = 0;
  return VSP_OK;
}

vsp_status vsp_profile_read(vsp_context* ctx, int which, double* total_ms, uint64_t* launches) {
  vsp_status s = check_ctx(ctx);
  if (s) return s;
  if (which < 0 || which >= kProfClasses || total_ms == nullptr || launches == nullptr)
    return fail(VSP_E_ARG, "which must be 0, 1, 2 or 3 and the outputs non-NULL");
  VSP_HIP(hipSetDevice(ctx->device));
  VSP_HIP(hipDeviceSynchronize());
  double t = 0;
  uint64_t n = 0;
  for (auto& p : ctx->prof.ev[which]) {
    float ms = 0;
    VSP_HIP(hipEventElapsedTime(&ms, p.e0, p.e1));
    t += ms;
    n += p.launches;
  }
  *total_ms = t;
  *launches = n;
  return VSP_OK;
}

vsp_status vsp_debug_external_product(vsp_context* ctx, const uint32_t* d_trgsw, const uint32_t* d_x,
                                      uint32_t* d_out, uint64_t J, void* stream) {
  vsp_status s = check_ctx(ctx);
  if (s) return s;
  if (J == 0) return VSP_OK;
  VSP_HIP(hipSetDevice(ctx->device));
  const size_t cb = (size_t)J * 2 * GADGET_L * 2 * RING_N * 4, xb = (size_t)J * 2 * RING_N * 4;
  if ((s = check_device_range(ctx, d_trgsw, cb, "d_trgsw"))) return s;
  if ((s = check_device_range(ctx, d_x, xb, "d_x"))) return s;
  if ((s = check_device_range(ctx, d_out, xb, "d_out"))) return s;
  if ((s = check_no_overlap(d_out, xb, d_x, xb, "d_out and d_x"))) return s;
  if ((s = check_no_overlap(d_out, xb, d_trgsw, cb, "d_out and d_trgsw"))) return s;
  if ((s = scratch_reserve(ctx, ctx->ntt_sel, (size_t)J * TRGSW_NTT_U64 * 8))) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint64_t* cn = static_cast<uint64_t*>(ctx->ntt_sel.ptr);
  hipError_t e;
  if ((e = launch_trgsw_to_ntt(ctx, d_trgsw, cn, J, st)) != hipSuccess) return hip_fail(e, "trgsw conversion");
  if ((e = launch_ext_product(ctx, cn, d_x, d_out, J, st)) != hipSuccess) return hip_fail(e, "external product");
  return VSP_OK;
}

vsp_status vsp_debug_polymul(vsp_context* ctx, const int32_t* d_a, const uint32_t* d_b, uint32_t* d_out, uint64_t J,
                             void* stream) {
  vsp_status s = check_ctx(ctx);
  if (s) return s;
  if (J == 0) return VSP_OK;
  VSP_HIP(hipSetDevice(ctx->device));
  const size_t b = (size_t)J * RING_N * 4;
  if ((s = check_device_range(ctx, d_a, b, "d_a"))) return s;
  if ((s = check_device_range(ctx, d_b, b, "d_b"))) return s;
  if ((s = check_device_range(ctx, d_out, b, "d_out"))) return s;
  if ((s = check_no_overlap(d_out, b, d_a, b, "d_out and d_a"))) return s;
  if ((s = check_no_overlap(d_out, b, d_b, b, "d_out and d_b"))) return s;
  hipError_t e = launch_polymul(ctx, d_a, d_b, d_out, J, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "polymul");
  return VSP_OK;
}

}  // extern "C"
