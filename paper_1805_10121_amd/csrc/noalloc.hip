// chase_filter_noalloc: the Chebyshev filter (Algorithm 4, Eq. (7)) for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops).  It runs the same
// products as chase_filter; the stream-K partial sums that chase_filter keeps in its context's
// scratch live here in a fixed device array, one per GPU, held until the process ends.
//
// The array is a file-scope __device__ symbol.  Host code never passes its name to a kernel:
// once per device, with that device current, its device address is looked up with
// hipGetSymbolAddress and kept, and only that address is handed to the kernels.  Nothing in the
// array has to start at zero: every partial-sum slot a fixup reads was written by the same
// filter product.  Calls that overlap on one GPU share the array and therefore race.

#include <cstdio>
#include <mutex>

#include "internal.h"

namespace {

// 96 MiB: the stream-K partial sums of every complex tile on a 256-CU device (the largest, the
// FP64 3M tile at three workgroups per CU, needs exactly this); the real FP64 128 x 128 tile
// (128 MiB there) is refused.
constexpr size_t kStaticScratchBytes = size_t{96} << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

struct DeviceScratch {
  void* ptr = nullptr;  // device address of this device's copy of `scratch`
  int cus = 0;
  bool ready = false;
};
DeviceScratch g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Fills ps with `device`'s scratch (looked up on the first call; the device must be current).
int device_scratch(chase_ctx* ctx, int device, chase::ProductScratch* ps) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  DeviceScratch& d = g_scratch[device];
  if (!d.ready) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return chase::set_error(ctx, CHASE_EDEVICE,
                              std::string("hipGetSymbolAddress of the static scratch: ") +
                                  hipGetErrorString(e));
    }
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess || cus <= 0) {
      (void)hipGetLastError();
      return chase::set_error(ctx, CHASE_EDEVICE, "cannot read the compute-unit count");
    }
    d.ptr = ptr;
    d.cus = cus;
    d.ready = true;
  }
  ps->ptr = d.ptr;
  ps->bytes = kStaticScratchBytes;
  ps->cus = d.cus;
  ps->sk_need = nullptr;
  return CHASE_OK;
}

int filter_noalloc(chase_ctx* ctx, int device, hipStream_t stream, int precision, const void* H,
                   int64_t ldh, int64_t n, void* V, void* W, int64_t ld, int64_t ncols,
                   const int32_t* degrees, double b_sup, double mu_1, double mu_nevnex) {
  using namespace chase;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(ctx, CHASE_EDEVICE, "no HIP device");
  }
  if (device < 0 || device >= count || device >= kMaxDevices)
    return set_error(ctx, CHASE_EINVAL, "device index out of range");
  if (precision == CHASE_FP64_LOWER)
    return set_error(ctx, CHASE_EINVAL, "CHASE_FP64_LOWER applies to chase_hemm_step only");
  int rc = check_product_args(ctx, precision, H, ldh, n, V, ld, W, ld, ncols);
  if (rc) return rc;
  CHASE_HIP_TRY(ctx, hipSetDevice(device));
  ProductScratch ps;
  if ((rc = device_scratch(ctx, device, &ps))) return rc;
  if (n == 0 || ncols == 0) return CHASE_OK;
  if ((rc = check_degrees(ctx, degrees, ncols))) return rc;
  if ((rc = check_bounds(ctx, b_sup, mu_1, mu_nevnex))) return rc;
  // Dry run: the largest stream-K partial-sum area any product of this call would use.
  size_t need = 0;
  ProductScratch dry = ps;
  dry.sk_need = &need;
  hipError_t e = run_filter_precision(precision, H, ldh, n, V, W, ld, ncols, degrees, b_sup, mu_1,
                                      mu_nevnex, dry, stream);
  if (e != hipSuccess)
    return set_error(ctx, CHASE_EDEVICE, std::string("filter plan: ") + hipGetErrorString(e));
  if (need > kStaticScratchBytes)
    return set_error(ctx, CHASE_EINVAL,
                     "this filter's stream-K schedule needs " + std::to_string(need) +
                         " bytes of partial-sum scratch; the static buffer holds " +
                         std::to_string(kStaticScratchBytes) + " bytes");
  e = run_filter_precision(precision, H, ldh, n, V, W, ld, ncols, degrees, b_sup, mu_1,
                           mu_nevnex, ps, stream);
  if (e != hipSuccess)
    return set_error(ctx, CHASE_EDEVICE, std::string("filter launch: ") + hipGetErrorString(e));
  return CHASE_OK;
}

}  // namespace

extern "C" int chase_filter_noalloc(int device, void* hip_stream, int precision, const void* H,
                                    int64_t ldh, int64_t n, void* V, void* W, int64_t ld,
                                    int64_t ncols, const int32_t* degrees, double b_sup,
                                    double mu_1, double mu_nevnex, char* err, size_t err_len) {
  chase_ctx msg;  // carries only the error text; no device resources
  const int rc = filter_noalloc(&msg, device, static_cast<hipStream_t>(hip_stream), precision, H,
                                ldh, n, V, W, ld, ncols, degrees, b_sup, mu_1, mu_nevnex);
  if (err && err_len > 0) std::snprintf(err, err_len, "%s", msg.last_error.c_str());
  return rc;
}
