// Autotuner for the batched launches. On random ciphertexts it times one full round of gates
// for each blind-rotation form (4 or 8 gates per workgroup at one wave per gate, one gate on
// three waves, and the matrix-core form; a launch then picks the form with the fewest rounds x
// round time for its batch), the split matrix-core form at thirteen batch sizes with each
// workgroup-group count (row groups or byte-plane ranges, atomics or partial sums; the fastest
// is kept per size) and the four key-switch forms (one workgroup per gate, row-stationary
// tiles, LDS-staged split, matrix cores) per batch-size bucket. Every candidate
// must produce bit-identical outputs. The result can be cached in a small JSON file keyed by
// the GPU; a cache written for another list of forms is ignored.
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "vsp_internal.h"

using namespace vsp;

namespace {

__global__ void k_fill_random(uint32_t* p, uint64_t n, uint64_t seed, uint32_t mod) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + i * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  p[i] = mod ? (uint32_t)(z % mod) : (uint32_t)z;
}

__global__ void k_u32_to_u8(const uint32_t* src, uint8_t* dst, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (uint8_t)src[i];
}

hipError_t fill(uint32_t* p, uint64_t n, uint64_t seed, uint32_t mod, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_random, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, seed, mod);
  return hipGetLastError();
}

std::string device_key(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string arch = p.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  return arch + "-" + std::to_string(p.multiProcessorCount) + "cu";
}

// Cache file: {"<device>": {"br_waves": [4, 8, ..], "br_cap": [..], "br_round_ms": [..],
//                          "buckets": [..], "ks_form": [..], "split_at": [..],
//                          "split_ms": [..], "split_groups": [..]}}
bool read_numbers(const std::string& s, size_t from, const char* name, double* out, int count) {
  const size_t p = s.find(std::string("\"") + name + "\"", from);
  if (p == std::string::npos) return false;
  const size_t lb = s.find('[', p);
  if (lb == std::string::npos) return false;
  const char* c = s.c_str() + lb + 1;
  for (int i = 0; i < count; i++) {
    char* end = nullptr;
    const double v = std::strtod(c, &end);
    if (end == c) return false;
    out[i] = v;
    c = end;
    while (*c == ',' || *c == ' ') c++;
  }
  return *c == ']';
}

bool read_cache(const std::string& path, const std::string& key, Tuning& t) {
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  const size_t at = s.find("\"" + key + "\"");
  if (at == std::string::npos) return false;
  double shapes[kBrShapes], cap[kBrShapes], ms[kBrShapes], ks[kTuneBuckets], buckets[kTuneBuckets];
  double sms[kSplitPts], sg[kSplitPts], spts[kSplitPts];
  if (!read_numbers(s, at, "br_waves", shapes, kBrShapes) || !read_numbers(s, at, "br_cap", cap, kBrShapes) ||
      !read_numbers(s, at, "br_round_ms", ms, kBrShapes) || !read_numbers(s, at, "buckets", buckets, kTuneBuckets) ||
      !read_numbers(s, at, "ks_form", ks, kTuneBuckets) || !read_numbers(s, at, "split_at", spts, kSplitPts) ||
      !read_numbers(s, at, "split_ms", sms, kSplitPts) || !read_numbers(s, at, "split_groups", sg, kSplitPts))
    return false;
  for (int i = 0; i < kBrShapes; i++)
    if (shapes[i] != kBrWaveChoices[i]) return false;  // written for another list of forms
  for (int b = 0; b < kTuneBuckets; b++)
    if (buckets[b] != (double)kBucket[b]) return false;
  Tuning n = t;  // keeps forced shapes
  for (int i = 0; i < kBrShapes; i++) {
    if (!(cap[i] >= 1 && cap[i] < 1e9 && ms[i] > 0 && ms[i] < 1e9)) return false;
    n.br_cap[i] = (uint64_t)cap[i];
    n.br_round_ms[i] = (float)ms[i];
  }
  for (int b = 0; b < kTuneBuckets; b++) {
    if (!(ks[b] >= 0 && ks[b] < kKsForms && ks[b] == (double)(int)ks[b])) return false;
    n.ks_form[b] = (int)ks[b];
  }
  for (int k = 0; k < kSplitPts; k++) {
    const int g = (int)sg[k];
    if (spts[k] != (double)kSplitAt[k]) return false;  // written for other sizes
    if (!(sms[k] > 0 && sms[k] < 1e9) || (double)g != sg[k] || !(g == 0 || split_groups_valid(g)))
      return false;
    n.split_ms[k] = (float)sms[k];
    n.split_groups[k] = g;
  }
  n.tuned = true;
  t = n;
  return true;
}

bool write_cache(const std::string& path, const std::string& key, const Tuning& t) {
  std::ofstream f(path, std::ios::trunc);
  if (!f) return false;
  auto list = [&](auto get, int count) {
    f << "[";
    for (int i = 0; i < count; i++) f << (i ? ", " : "") << get(i);
    f << "]";
  };
  f << "{\"" << key << "\": {\"br_waves\": ";
  list([](int i) { return kBrWaveChoices[i]; }, kBrShapes);
  f << ", \"br_cap\": ";
  list([&](int i) { return t.br_cap[i]; }, kBrShapes);
  f << ", \"br_round_ms\": ";
  list([&](int i) { return t.br_round_ms[i]; }, kBrShapes);
  f << ", \"buckets\": ";
  list([](int i) { return kBucket[i]; }, kTuneBuckets);
  f << ", \"ks_form\": ";
  list([&](int i) { return t.ks_form[i]; }, kTuneBuckets);
  f << ", \"split_at\": ";
  list([](int i) { return kSplitAt[i]; }, kSplitPts);
  f << ", \"split_ms\": ";
  list([&](int i) { return t.split_ms[i]; }, kSplitPts);
  f << ", \"split_groups\": ";
  list([&](int i) { return t.split_groups[i]; }, kSplitPts);
  f << "}}\n";
  return (bool)f;
}

struct Buf {
  void* p = nullptr;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

extern "C" {

vsp_status vsp_autotune(vsp_context* ctx, uint64_t max_batch, const char* cache_path) {
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  if (max_batch == 0 || max_batch > (1ull << 20)) return fail(VSP_E_ARG, "max_batch must be in [1, 2^20]");
  VSP_HIP(hipSetDevice(ctx->device));
  const std::string key = device_key(ctx->device);
  if (cache_path && read_cache(cache_path, key, ctx->tune)) return VSP_OK;

  const uint64_t Sks = std::min<uint64_t>(max_batch, kBucket[kTuneBuckets - 1]);
  uint64_t Sbr = 0;
  for (int s = 0; s < kBrShapes; s++) Sbr = std::max(Sbr, ctx->tune.br_cap[s]);
  const uint64_t S = std::max(Sks, Sbr);
  Buf in, ops32, ops, abar, t1, t1ref, out, outref;
  const size_t T0 = (LWE_N + 1) * 4, T1 = (RING_N + 1) * 4;
  VSP_HIP(hipMalloc(&in.p, 2 * S * T0));
  VSP_HIP(hipMalloc(&ops32.p, S * 4));
  VSP_HIP(hipMalloc(&ops.p, S));
  VSP_HIP(hipMalloc(&abar.p, S * T0));
  VSP_HIP(hipMalloc(&t1.p, S * T1));
  VSP_HIP(hipMalloc(&t1ref.p, S * T1));
  VSP_HIP(hipMalloc(&out.p, S * T0));
  VSP_HIP(hipMalloc(&outref.p, S * T0));
  hipStream_t st = nullptr;
  uint32_t* i0 = static_cast<uint32_t*>(in.p);
  uint32_t* i1 = i0 + S * (LWE_N + 1);
  hipError_t e;
  if ((e = fill(i0, 2 * S * (LWE_N + 1), 0x5eed, 0, st)) != hipSuccess) return hip_fail(e, "fill");
  if ((e = fill(static_cast<uint32_t*>(ops32.p), S, 0x0b5, 8, st)) != hipSuccess) return hip_fail(e, "fill");
  hipLaunchKernelGGL(k_u32_to_u8, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, st,
                     static_cast<const uint32_t*>(ops32.p), static_cast<uint8_t*>(ops.p), S);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "ops");
  const uint8_t* dops = static_cast<const uint8_t*>(ops.p);
  uint32_t* dab = static_cast<uint32_t*>(abar.p);
  if ((e = launch_gate_prologue(ctx, dops, i0, i1, nullptr, nullptr, nullptr, dab, static_cast<uint32_t*>(out.p), S,
                                st)) != hipSuccess)
    return hip_fail(e, "prologue");
  hipEvent_t ev0, ev1;
  VSP_HIP(hipEventCreate(&ev0));
  VSP_HIP(hipEventCreate(&ev1));
  auto timed = [&](auto&& launch) -> float {
    launch();  // warm
    (void)hipEventRecord(ev0, st);
    launch();
    (void)hipEventRecord(ev1, st);
    (void)hipEventSynchronize(ev1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    return ms;
  };
  std::vector<uint32_t> ha, hb;
  auto same = [&](const void* a, const void* b, size_t bytes) {
    ha.resize(bytes / 4);
    hb.resize(bytes / 4);
    (void)hipMemcpy(ha.data(), a, bytes, hipMemcpyDeviceToHost);
    (void)hipMemcpy(hb.data(), b, bytes, hipMemcpyDeviceToHost);
    return std::memcmp(ha.data(), hb.data(), bytes) == 0;
  };
  Tuning t = ctx->tune;
  vsp_status result = VSP_OK;
  // Blind rotation: one full round of gates per shape.
  if (ctx->mf_key && (result = scratch_reserve(ctx, ctx->mf_work, mf_work_bytes(t.br_cap[3], true))) != VSP_OK)
    return result;
  for (int s = 0; s < kBrShapes && result == VSP_OK; s++) {
    uint32_t* dst = static_cast<uint32_t*>(s == 0 ? t1ref.p : t1.p);
    const uint64_t B = t.br_cap[s];
    t.br_round_ms[s] = timed([&] {
      (void)launch_blind_rotate(ctx, dops, dab, dst, nullptr, B, kBrWaveChoices[s], st, nullptr, nullptr, nullptr,
                                ctx->mf_work.ptr);
    });
    if (s > 0 && !same(t1ref.p, t1.p, std::min(t.br_cap[0], B) * T1))
      result = fail(VSP_E_HIP, "autotune: blind-rotation shapes disagree");
  }
  // the split matrix-core form at each timed size, with each workgroup count
  for (int b = 0; b < kSplitPts && result == VSP_OK && ctx->mf_key; b++) {
    const uint64_t B = std::min<uint64_t>(kSplitAt[b], t.br_cap[3]);
    float best = 1e30f;
    for (int g : kSplitGroupChoices) {
      if ((g > 6 || g < -6) && B > 256) continue;  // plane ranges (12, 24) only pay while tiles are few
      if (g < 0 && B < 16) continue;   // partial sums only pay once atomics pile up
      const float ms = timed([&] {
        (void)launch_blind_rotate_mfsplit(ctx, dops, dab, static_cast<uint32_t*>(t1.p), nullptr, B, ctx->mf_work.ptr,
                                          g, st);
      });
      if (!same(t1ref.p, t1.p, std::min(t.br_cap[0], B) * T1))
        result = fail(VSP_E_HIP, "autotune: blind-rotation shapes disagree");
      if (ms < best) {
        best = ms;
        t.split_ms[b] = ms;
        t.split_groups[b] = g;
      }
    }
  }
  // Key switch on random TLWE1 rows, per bucket, at the bucket's largest batch.
  if (result == VSP_OK && (e = fill(static_cast<uint32_t*>(t1ref.p), S * (RING_N + 1), 0x7a11, 0, st)) != hipSuccess)
    result = hip_fail(e, "fill");
  for (int b = 0; b < kTuneBuckets && result == VSP_OK; b++) {
    if (b > 0 && kBucket[b - 1] >= Sks) {  // beyond the batches asked for: keep the previous choice
      t.ks_form[b] = t.ks_form[b - 1];
      continue;
    }
    const uint64_t B = std::min<uint64_t>(kBucket[b], Sks);
    float best = 1e30f;
    for (int c = 0; c < kKsForms && result == VSP_OK; c++) {
      uint32_t* dst = static_cast<uint32_t*>(c == 0 ? outref.p : out.p);
      const float ms = timed([&] { (void)launch_keyswitch(ctx, dops, static_cast<const uint32_t*>(t1ref.p), nullptr,
                                                          dst, B, st, c); });
      if (c > 0 && !same(outref.p, out.p, B * T0)) result = fail(VSP_E_HIP, "autotune: key-switch forms disagree");
      if (ms < best) {
        best = ms;
        t.ks_form[b] = c;
      }
    }
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "autotune");
  if (result != VSP_OK) return result;
  t.tuned = true;
  ctx->tune = t;
  if (cache_path && !write_cache(cache_path, key, t)) return fail(VSP_E_ARG, "cannot write the autotune cache file");
  return VSP_OK;
}

vsp_status vsp_tuning_get(const vsp_context* ctx, uint64_t B, int* br_waves, int* ks_form) {
  if (ctx == nullptr || br_waves == nullptr || ks_form == nullptr) return fail(VSP_E_ARG, "NULL argument");
  *br_waves = ctx->tune.br_waves(B == 0 ? 1 : B);
  *ks_form = ctx->tune.ks_form_for(B == 0 ? 1 : B);
  return VSP_OK;
}

vsp_status vsp_tuning_set_split(vsp_context* ctx, uint64_t B, int groups, int* previous) {
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  if (groups != 0 && !split_groups_valid(groups))
    return fail(VSP_E_ARG, "groups must be 0 (the count that fills the chip), 1, 2, 3, 6, 12, 24, -1, -2, -3, -6, -12 or -24");
  const int k = Tuning::split_point(B == 0 ? 1 : B);
  if (previous) *previous = ctx->tune.split_groups[k];
  ctx->tune.split_groups[k] = groups;
  return VSP_OK;
}

vsp_status vsp_tuning_set(vsp_context* ctx, uint64_t B, int br_waves, int ks_form) {
  if (ctx == nullptr) return fail(VSP_E_ARG, "context is NULL");
  if ((br_waves != 0 && br_waves != 3 && br_waves != 4 && br_waves != 8 && br_waves != 32 && br_waves != 33) ||
      ks_form < 0 || ks_form >= kKsForms)
    return fail(VSP_E_ARG, "br_waves must be 0 (model), 3, 4, 8, 32 or 33 and ks_form 0, 1, 2 or 3");
  const int b = Tuning::bucket(B == 0 ? 1 : B);
  ctx->tune.br_force[b] = br_waves;
  ctx->tune.ks_form[b] = ks_form;
  return VSP_OK;
}

}  // extern "C"
