// tgks_noalloc.hip -- one S2O4 step that allocates nothing
// (tgks_step_noalloc, include/tgks.h).
//
// The step's work buffers (W*, the accumulator P, the face flux arrays, the
// 3-D normal reconstruction, CFL partial minima, the clock and the failure
// counters) live in one file-scope device array instead of a context's
// allocations.  Each GPU holds its own copy of the array until the process
// ends; its device address is looked up once per device and kept.  Calls
// that overlap on one GPU share the array and race.
#include <mutex>

#include "tgks_internal.hpp"

namespace {

constexpr long long SCRATCH_DOUBLES = 8LL << 20;  // 64 MiB
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

double* scratch_dev[MAX_DEVICES];  // device address of `scratch` per device
std::mutex scratch_mtx;

// the device address of this device's copy of the array (looked up on the
// first call with the device current)
int scratch_of_current(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return TGKS_EHIP;
  std::lock_guard<std::mutex> lock(scratch_mtx);
  if (!scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      fprintf(stderr, "tgks: hipGetSymbolAddress(scratch) failed: %s\n", hipGetErrorString(e));
      return TGKS_EHIP;
    }
    scratch_dev[dev] = static_cast<double*>(ptr);
  }
  *out = scratch_dev[dev];
  return TGKS_OK;
}

// doubles of a region rounded up to 256 bytes
inline long long pad(long long n) { return (n + 31) / 32 * 32; }

}  // namespace

extern "C" {

int64_t tgks_noalloc_capacity(void) { return SCRATCH_DOUBLES; }

int64_t tgks_noalloc_need(const tgks_params* p) {
  if (check_params(p)) return TGKS_EINVAL;
  tgks_ctx c;
  init_ctx_host(&c, p, nullptr);
  long long need = 2 * pad((long long)c.nc * c.ncell);
  for (int d = 0; d < c.g.D; ++d) need += 2 * pad((long long)c.nc * c.nface[d]);
  if (c.g.D == 3) {
    long long mx = 0;
    for (int d = 0; d < 3; ++d) {
      long long nr = 1;
      for (int e = 0; e < 3; ++e) nr *= (long long)(c.g.n[e] + 2 * (e == d));
      mx = nr > mx ? nr : mx;
    }
    need += pad(mx * 4 * 5);
  }
  need += pad(c.nblk) + pad(4) + pad(2);
  return need;
}

int tgks_step_noalloc(const tgks_params* p, void* hip_stream, const double* W_in, double* W_out,
                      const double* dt_dev, uint8_t* flags, double* W_star, int64_t* failures) {
  if (check_params(p) || !W_in || !W_out || !dt_dev || W_in == W_out) return TGKS_EINVAL;
  const int64_t need = tgks_noalloc_need(p);
  if (need < 0 || need > SCRATCH_DOUBLES) {
    fprintf(stderr, "tgks: tgks_step_noalloc needs %lld doubles of scratch, the maximum is %lld\n",
            (long long)need, SCRATCH_DOUBLES);
    return TGKS_EINVAL;
  }
  double* base = nullptr;
  int r = scratch_of_current(&base);
  if (r) return r;
  // a context on the host stack whose buffers are regions of the array
  tgks_ctx c;
  init_ctx_host(&c, p, hip_stream);
  double* q = base;
  auto take = [&q](long long n) {
    double* o = q;
    q += pad(n);
    return o;
  };
  c.Ws = take((long long)c.nc * c.ncell);
  c.P = take((long long)c.nc * c.ncell);
  for (int d = 0; d < c.g.D; ++d) {
    c.FA[d] = take((long long)c.nc * c.nface[d]);
    c.FB[d] = take((long long)c.nc * c.nface[d]);
  }
  if (c.g.D == 3) {
    long long mx = 0;
    for (int d = 0; d < 3; ++d) {
      long long nr = 1;
      for (int e = 0; e < 3; ++e) nr *= (long long)(c.g.n[e] + 2 * (e == d));
      mx = nr > mx ? nr : mx;
    }
    c.R = take(mx * 4 * 5);
  }
  c.partial = take(c.nblk);
  c.clock = take(4);
  c.fail = reinterpret_cast<unsigned long long*>(take(2));
  // the counters keep the last call's values: clear them (a kernel, so that
  // the call may be captured into a graph)
  hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(256), 0, c.stream, c.fail, 2);
  HIPCHK(hipGetLastError());
  if ((r = do_step(&c, W_in, W_out, dt_dev, flags, false))) return r;
  if (W_star)
    HIPCHK(hipMemcpyAsync(W_star, c.Ws, (size_t)c.nc * c.ncell * sizeof(double), hipMemcpyDeviceToDevice,
                          c.stream));
  if (failures) {
    unsigned long long f = 0;
    HIPCHK(hipMemcpyAsync(&f, c.fail, sizeof(f), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    *failures = (int64_t)f;
  }
  return TGKS_OK;
}

}  // extern "C"
