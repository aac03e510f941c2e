// Streaming probes of the device's HBM: the bandwidth a plain float4 stream
// reaches, the denominator of the "fraction of what the memory system
// delivers" beside the 8 TB/s nominal peak.  Grid-stride loops of 256-thread
// blocks over float4 elements:
//   copy   dst[i] = src[i]           (bytes read + bytes written)
//   read   sum of src, one float per block into dst (bytes read)
//   write  dst[i] = constant, non-temporal stores (bytes written)
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lbm.h"

namespace {

__global__ void __launch_bounds__(256)
    k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x)
    dst[i] = src[i];
}

__global__ void __launch_bounds__(256)
    k_probe_read(const float4* __restrict__ src, float* __restrict__ out, long long n) {
  float acc = 0.0f;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const float4 v = src[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  __shared__ float sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

typedef float vf4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_probe_write(float4* __restrict__ dst, long long n) {
  const vf4 v = {1.0f, 2.0f, 3.0f, 4.0f};
  vf4* d = reinterpret_cast<vf4*>(dst);
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x)
    __builtin_nontemporal_store(v, d + i);
}

thread_local char g_probe_err[256];

int probe_fail(const char* what, hipError_t e) {
  const char* msg = e == hipSuccess ? "" : hipGetErrorString(e);
  int i = 0;
  for (const char* p = what; *p && i < 200; ++p) g_probe_err[i++] = *p;
  g_probe_err[i++] = ' ';
  for (const char* p = msg; *p && i < 254; ++p) g_probe_err[i++] = *p;
  g_probe_err[i] = '\0';
  return e == hipSuccess ? LBM_EINVAL : LBM_EDEVICE;
}

}  // namespace

extern "C" int lbm_bandwidth_probe(int kind, void* dst_dev, const void* src_dev, int64_t bytes,
                                   int blocks, int iters, void* stream, double* gbs_out) {
  if (kind < 0 || kind > 2) return probe_fail("kind must be 0 (copy), 1 (read) or 2 (write)",
                                              hipSuccess);
  if (bytes < 16 || bytes % 16 != 0) return probe_fail("bytes must be a positive multiple of 16",
                                                       hipSuccess);
  if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > 10000)
    return probe_fail("blocks must be in 1..2^20 and iters in 1..10000", hipSuccess);
  if (!dst_dev || (kind != 2 && !src_dev) || !gbs_out)
    return probe_fail("null buffer or output", hipSuccess);
  const auto st = static_cast<hipStream_t>(stream);
  const long long n = bytes / 16;
  auto launch = [&]() {
    if (kind == 0)
      hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, st,
                         static_cast<const float4*>(src_dev), static_cast<float4*>(dst_dev), n);
    else if (kind == 1)
      hipLaunchKernelGGL(k_probe_read, dim3(blocks), dim3(256), 0, st,
                         static_cast<const float4*>(src_dev), static_cast<float*>(dst_dev), n);
    else
      hipLaunchKernelGGL(k_probe_write, dim3(blocks), dim3(256), 0, st,
                         static_cast<float4*>(dst_dev), n);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    launch();  // warm-up
    e = hipEventRecord(e0, st);
  }
  for (int i = 0; i < iters && e == hipSuccess; ++i) {
    launch();
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return probe_fail("probe", e);
  const double moved = static_cast<double>(bytes) * (kind == 0 ? 2.0 : 1.0);
  *gbs_out = moved * iters / (ms / 1e3) / 1e9;
  return LBM_OK;
}

extern "C" const char* lbm_probe_last_error(void) { return g_probe_err; }
