// closure_moments without a workspace: the per-chunk partial sums live in a
// file-scope device array, for callers that cannot allocate device memory
// (code under graph capture, serving loops).
//
// Each GPU holds its own copy of the array; its address is looked up once
// per device with hipGetSymbolAddress, with that device current, and the
// kernels receive that address. Every call on a device shares its array:
// calls that overlap on one GPU (two streams, or two threads) race.
#include <mutex>

#include "eles.h"
#include "eles_internal.h"

namespace {

// chunks per channel, as closure_moments
constexpr int kChunks = 1024;
static_assert((size_t)ELES_MOMENTS_NOALLOC_MAX_CHAN * kChunks * sizeof(double) <= (512u << 10),
              "scratch of the no-workspace moments stays at 512 KiB");

static __device__ __align__(256) double scratch[ELES_MOMENTS_NOALLOC_MAX_CHAN * kChunks];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch`.
hipError_t scratch_on_current_device(double **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = (double *)p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int32_t closure_moments_noalloc(const float *data, int32_t nchan, int32_t nsnap, int64_t npts,
                                           double *out, hipStream_t stream) {
  if (!data || !out || nchan < 1 || nsnap < 1 || npts < 1) return ELES_EINVAL;
  if (nchan > ELES_MOMENTS_NOALLOC_MAX_CHAN) return ELES_ENOSPACE;
  double *part = nullptr;
  if (scratch_on_current_device(&part) != hipSuccess) return ELES_EHIP;
  // every partial the final sums read is written first by the same call,
  // so the array needs no clearing between calls
  return eles::launch_moments(data, nchan, nsnap, (long)npts, part, kChunks, out, stream) == hipSuccess
             ? ELES_OK
             : ELES_EHIP;
}
