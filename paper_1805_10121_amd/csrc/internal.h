// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/chase.h"

namespace chase {

// Partial-sum scratch of the stream-K product schedule (owned by the context, fixed size).
struct ProductScratch {
  void* ptr = nullptr;
  size_t bytes = 0;
  int cus = 0;  // compute units of the device
};
size_t product_scratch_bytes(int cus);

// ----------------------------------------------------------------------------- kernels
// One fused complex product  OUT <- alpha*H*X + gamma*X + beta*OUT  on ncols columns.
// T = double (complex128 data) or float (complex64 data); pointers address interleaved
// (re, im) pairs, leading dimensions count complex elements.
template <typename T>
hipError_t launch_hemm_step(const T* H, int64_t ldh, int64_t n, const T* X, int64_t ldx, T* OUT,
                            int64_t ldo, int64_t ncols, T alpha, T beta, T gamma,
                            const ProductScratch& ps, hipStream_t stream);

hipError_t launch_convert_c128_to_c64(const double* src, int64_t lds, float* dst, int64_t ldd,
                                      int64_t rows, int64_t cols, hipStream_t stream);
hipError_t launch_convert_c64_to_c128(const float* src, int64_t lds, double* dst, int64_t ldd,
                                      int64_t rows, int64_t cols, hipStream_t stream);

// Outer-loop helpers (loop_kernels.hip); complex128 data as interleaved doubles.
hipError_t launch_lanczos_step(const double* U, const double* Up, double* W, double* Un, int64_t n,
                               int64_t ld, int64_t nv, const double* beta_prev, double* alpha_out,
                               double* beta_out, hipStream_t s);
hipError_t launch_normalize(double* X, int64_t n, int64_t ld, int64_t cols, hipStream_t s);
hipError_t launch_resid(const double* AV, const double* V, const double* lam, int64_t n, int64_t ld,
                        int64_t cols, double* out, hipStream_t s);
hipError_t launch_gather(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                         const int* perm, int64_t cols, hipStream_t s);
hipError_t launch_herm_sym(double* G, int64_t ld, int64_t m, hipStream_t s);
hipError_t launch_add_diag(double* G, int64_t ld, int64_t m, double v, hipStream_t s);
hipError_t launch_gaussian(double* X, int64_t n, int64_t ld, int64_t cols, uint64_t seed,
                           hipStream_t s);

// ----------------------------------------------------------------------------- filter driver
// Algorithm 4 on an n x ncols block with sorted even degrees (validated by the caller).  The
// result ends in V.  scalars: the per-product (alpha, beta, gamma) in FP64.
template <typename T>
hipError_t run_filter(const T* H, int64_t ldh, int64_t n, T* V, T* W, int64_t ld, int64_t ncols,
                      const int32_t* degrees, double b_sup, double mu_1, double mu_nevnex,
                      const ProductScratch& ps, hipStream_t stream, int64_t* matvecs_out);

}  // namespace chase

struct chase_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  rocblas_handle blas = nullptr;
  chase::ProductScratch prod;
  std::string last_error;
  // device workspace, grown monotonically
  void* ws = nullptr;
  size_t ws_bytes = 0;
};

namespace chase {
int set_error(chase_ctx* ctx, int code, const std::string& msg);
int ensure_workspace(chase_ctx* ctx, size_t bytes);
int hip_ok(chase_ctx* ctx);  // hipSetDevice(ctx->device) with error reporting
}  // namespace chase

#define CHASE_HIP_TRY(ctx, expr)                                                            \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return ::chase::set_error((ctx), CHASE_EDEVICE,                                       \
                                std::string(#expr) + ": " + hipGetErrorString(_e));         \
  } while (0)
