// tgks_peaks.hip -- the two ceilings of the roofline measured on the device
// the library runs on: FP64 fused multiply-add throughput (eight independent
// FMA chains per thread, enough waves to fill every SIMD) and device-to-
// device copy bandwidth (16-byte loads and stores over a 1 GiB buffer).
#include "tgks_internal.hpp"

namespace {

__global__ __launch_bounds__(256) void peak_fma_kernel(double* out, int iters, double x, double y) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  double a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = 1.0 + 1e-3 * (gid + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = fma(a[k], x, y);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  out[gid] = s;
}

__global__ __launch_bounds__(256) void copy_kernel(const double2* __restrict__ src, double2* __restrict__ dst,
                                                   long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" int tgks_measure_peaks(void* stream, double* fp64_tflops, double* copy_gbps) {
  if (!fp64_tflops || !copy_gbps) return TGKS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, ncu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const long long bytes = 1LL << 30;
  const int blocks = ncu * 32, threads = 256, iters = 4096;
  double* buf = nullptr;
  double* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = TGKS_OK;
  if (hipMalloc(&buf, 2 * bytes) != hipSuccess || hipMalloc(&out, (size_t)blocks * threads * sizeof(double)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = TGKS_EHIP;
  float ms = 0.f;
  if (!rc) {
    // FMA throughput: warm-up, then the timed launch
    hipLaunchKernelGGL(peak_fma_kernel, dim3(blocks), dim3(threads), 0, s, out, 64, 0.999999, 1e-7);
    (void)hipEventRecord(e0, s);
    hipLaunchKernelGGL(peak_fma_kernel, dim3(blocks), dim3(threads), 0, s, out, iters, 0.999999, 1e-7);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = TGKS_EHIP;
    if (!rc) *fp64_tflops = 2.0 * 8.0 * iters * (double)blocks * threads / (ms * 1e-3) / 1e12;
  }
  if (!rc) {
    // copy bandwidth: bytes read + bytes written
    const long long n = bytes / (long long)sizeof(double2);
    const double2* src = (const double2*)buf;
    double2* dst = (double2*)(buf + bytes / sizeof(double));
    (void)hipMemsetAsync(buf, 0, 2 * bytes, s);
    hipLaunchKernelGGL(copy_kernel, dim3(ncu * 16), dim3(256), 0, s, src, dst, n);
    (void)hipEventRecord(e0, s);
    hipLaunchKernelGGL(copy_kernel, dim3(ncu * 16), dim3(256), 0, s, src, dst, n);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = TGKS_EHIP;
    if (!rc) *copy_gbps = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  (void)hipFree(out);
  return rc;
}
