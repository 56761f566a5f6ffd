// Register-resident throughput of the arithmetic modulo p = 2^64 - 2^32 + 1 that the NTT form
// of the blind rotation is built from: the general product (gl_mul) and the lazy sum (gl_add),
// each in eight independent chains per lane at full occupancy, no memory traffic inside the
// loop. Their rates are the integer-VALU ceiling against which the method's own work per gate
// (products and sums modulo p of its transforms and key products) is priced.
#include "vsp_internal.h"

namespace vsp {

constexpr int kAluChains = 8;
constexpr int kAluThreads = 256;

__global__ __launch_bounds__(kAluThreads) void k_alu_mulmod(const u64* __restrict__ seed, u64* __restrict__ out,
                                                           uint32_t iters) {
  const uint64_t id = (uint64_t)blockIdx.x * kAluThreads + threadIdx.x;
  u64 x[kAluChains], y[kAluChains];
#pragma unroll
  for (int k = 0; k < kAluChains; k++) {
    x[k] = seed[k] + id;
    y[k] = seed[kAluChains + k] ^ (id << 7);
  }
  for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
    for (int k = 0; k < kAluChains; k++) x[k] = gl_mul(x[k], y[k]);
  }
  u64 r = 0;
#pragma unroll
  for (int k = 0; k < kAluChains; k++) r ^= x[k];
  out[id] = r;
}

__global__ __launch_bounds__(kAluThreads) void k_alu_addmod(const u64* __restrict__ seed, u64* __restrict__ out,
                                                           uint32_t iters) {
  const uint64_t id = (uint64_t)blockIdx.x * kAluThreads + threadIdx.x;
  u64 x[kAluChains], y[kAluChains];
#pragma unroll
  for (int k = 0; k < kAluChains; k++) {
    x[k] = seed[k] + id;
    y[k] = seed[kAluChains + k] ^ (id << 7);
  }
  for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
    for (int k = 0; k < kAluChains; k++) x[k] = gl_add(x[k], y[k]);
  }
  u64 r = 0;
#pragma unroll
  for (int k = 0; k < kAluChains; k++) r ^= x[k];
  out[id] = r;
}

}  // namespace vsp

using namespace vsp;

extern "C" {

vsp_status vsp_measure_modp(int device, uint32_t iters, double* mulmod_per_s, double* addmod_per_s) {
  if (mulmod_per_s == nullptr || addmod_per_s == nullptr) return fail(VSP_E_ARG, "outputs must not be NULL");
  if (iters < 16 || iters > (1u << 24)) return fail(VSP_E_ARG, "iters must be in [16, 2^24]");
  int ndev = 0;
  VSP_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(VSP_E_ARG, "no such device");
  VSP_HIP(hipSetDevice(device));
  int cus = 0, per_cu = 0;
  VSP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  VSP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_alu_mulmod),
                                                       kAluThreads, 0));
  if (per_cu < 1) per_cu = 1;
  // four full rounds of resident workgroups
  const uint64_t blocks = (uint64_t)cus * per_cu * 4;
  const uint64_t threads = blocks * kAluThreads;
  u64* seed = nullptr;
  u64* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  vsp_status st = VSP_OK;
  auto done = [&](vsp_status s) {
    if (seed) (void)hipFree(seed);
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return s;
  };
  hipError_t e;
  if ((e = hipMalloc(&seed, 2 * kAluChains * 8)) != hipSuccess) return done(hip_fail(e, "hipMalloc(seed)"));
  if ((e = hipMalloc(&out, threads * 8)) != hipSuccess) return done(hip_fail(e, "hipMalloc(out)"));
  u64 hs[2 * kAluChains];
  for (int k = 0; k < 2 * kAluChains; k++) hs[k] = 0x9E3779B97F4A7C15ull * (uint64_t)(k + 1) % GL_P;
  if ((e = hipMemcpy(seed, hs, sizeof(hs), hipMemcpyHostToDevice)) != hipSuccess) return done(hip_fail(e, "seed"));
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    return done(hip_fail(e, "hipEventCreate"));
  double rate[2] = {0, 0};
  for (int which = 0; which < 2 && st == VSP_OK; which++) {
    auto launch = [&] {
      if (which == 0)
        hipLaunchKernelGGL(k_alu_mulmod, dim3((unsigned)blocks), dim3(kAluThreads), 0, nullptr, seed, out, iters);
      else
        hipLaunchKernelGGL(k_alu_addmod, dim3((unsigned)blocks), dim3(kAluThreads), 0, nullptr, seed, out, iters);
    };
    launch();  // warm-up
    if ((e = hipEventRecord(e0, nullptr)) != hipSuccess) return done(hip_fail(e, "hipEventRecord"));
    launch();
    if ((e = hipEventRecord(e1, nullptr)) != hipSuccess) return done(hip_fail(e, "hipEventRecord"));
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return done(hip_fail(e, "modp benchmark"));
    float ms = 0;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return done(hip_fail(e, "hipEventElapsedTime"));
    rate[which] = (double)threads * kAluChains * iters / (ms * 1e-3);
  }
  *mulmod_per_s = rate[0];
  *addmod_per_s = rate[1];
  return done(VSP_OK);
}

}  // extern "C"
