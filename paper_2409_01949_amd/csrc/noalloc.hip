// x = M^T u without any device allocation, for callers that cannot allocate (code under HIP
// graph capture, serving loops, harnesses that forbid hipMalloc).
//
// elmfb_rmatvec keeps the per-chunk partial sums of its first pass in workspace the handle
// allocated.  This variant keeps them in `scratch`, a file-scope device array of fixed size that
// every GPU the library runs on holds until the process ends; the kernels are the same ones, so
// the result is bit-identical.  Host code never hands the array's name to a kernel or a copy:
// in host code that name is a host-side stand-in, so each device's address of the array is
// looked up once (hipGetSymbolAddress, with that device current) and kept per device.
#include <mutex>

#include "handle.h"

namespace {

// chunk partials: one double per (chunk of <= kChunkPts points, feature)
constexpr int64_t kNoAllocScratchDoubles = int64_t(1) << 18;   // 2 MiB
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kNoAllocScratchDoubles];

std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up on the first call there.
hipError_t scratch_for_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

}  // namespace

namespace elmfb {

// Called by elmfb_define_problem with the handle's device current, so the lookup happens at
// set-up and not inside a caller's captured or allocation-free region.
hipError_t noalloc_init_device() {
  double* p = nullptr;
  return scratch_for_current_device(&p);
}

}  // namespace elmfb

extern "C" elmfb_status elmfb_rmatvec_noalloc(elmfb_problem h, const double* u_dev,
                                              double* x_dev, void* stream) {
  if (!h || !u_dev || !x_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "rmatvec_noalloc before assemble");
  const Geo& g = h->geo;
  const int64_t need = (int64_t)h->chunks.size() * g.K;
  if (need > kNoAllocScratchDoubles)
    return fail(h, ELMFB_E_UNSUPPORTED,
                "rmatvec_noalloc: " + std::to_string(need) + " chunk partials exceed the " +
                    std::to_string(kNoAllocScratchDoubles) +
                    " of the library's fixed scratch array; use elmfb_rmatvec");
  double* part = nullptr;
  HIP_OR_FAIL(h, scratch_for_current_device(&part));
  hipStream_t s = (hipStream_t)stream;
  // every chunk writes all K of its partials before the column pass reads them: nothing in the
  // array has to start at zero
  HIP_OR_FAIL(h, launch_rmv_chunks(g, ELMFB_FP64, h->d_blocks, h->d_chunks,
                                   (int64_t)h->chunks.size(), h->d_A, u_dev, nullptr, part,
                                   nullptr, s));
  // COL_STORE writes no norm partials, so the handle's reduction workspace is not touched
  HIP_OR_FAIL(h, launch_rmv_finish(g, h->d_cstart, part, COL_STORE, x_dev, nullptr, nullptr,
                                   cols_wg(g), h->d_bc, u_dev, nullptr, s));
  return ELMFB_OK;
}
