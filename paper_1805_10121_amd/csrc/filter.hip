// Host side of the Chebyshev filter (Algorithm 4 with the scaled recurrence of Eq. (7)), for
// complex Hermitian H (4M or 3M products, FP32 or FP64) and real symmetric H (kind 3, real
// products).
//
// The coefficients are scalars computed here in FP64 and passed to each launch:
//   product 1:   W <- (sigma_1/e) (H - cI) V                      (Alg. 4, first step)
//   product i>1: V[:, s:] <- (2 tau/e)(H - cI) W[:, s:] - tau sigma V[:, s:], swap V, W   (recurrence)
// with sigma_1 = e/(mu_1 - c), tau = 1/(2/sigma_1 - sigma) and sigma <- tau.  The active range
// starts at s, the first column whose degree exceeds the products done so far (Alg. 4's active range);
// degrees are sorted, so the range is a contiguous suffix and one launch covers it.

#include "internal.h"

namespace chase {

template <typename T>
hipError_t run_filter(const T* H, int64_t ldh, int64_t n, T* V, T* W, int64_t ld, int64_t ncols,
                      const int32_t* degrees, double b_sup, double mu_1, double mu_nevnex,
                      const ProductScratch& ps, hipStream_t stream, int64_t* matvecs_out,
                      int kind) {
  int64_t matvecs = 0;
  const int ew = kind == 3 ? 1 : 2;  // values per element
  hipError_t status = hipSuccess;
  if (ncols > 0 && n > 0) {
    for_each_filter_product(ncols, degrees, b_sup, mu_1, mu_nevnex, [&](const FilterProduct& p) {
      if (status != hipSuccess) return;
      const T* X = (p.from_v ? V : W) + ew * p.col0 * ld;
      T* OUT = (p.from_v ? W : V) + ew * p.col0 * ld;
      hipError_t err;
      if (kind == 3) {
        err = launch_hemm_step_real<T>(H, ldh, n, X, ld, OUT, ld, p.ncols, static_cast<T>(p.alpha),
                                       static_cast<T>(p.beta), static_cast<T>(p.gamma), ps, stream);
      } else if constexpr (sizeof(T) == 4) {
        if (kind == 2)
          err = launch_hemm_step_3m(H, ldh, n, X, ld, OUT, ld, p.ncols, static_cast<T>(p.alpha),
                                    static_cast<T>(p.beta), static_cast<T>(p.gamma), ps, stream);
        else
          err = launch_hemm_step<T>(H, ldh, n, X, ld, OUT, ld, p.ncols, static_cast<T>(p.alpha),
                                    static_cast<T>(p.beta), static_cast<T>(p.gamma), ps, stream);
      } else if (kind == 4) {
        err = launch_hemm_step_3m_f64(H, ldh, n, X, ld, OUT, ld, p.ncols, p.alpha, p.beta,
                                      p.gamma, ps, stream);
      } else {
        err = launch_hemm_step<T>(H, ldh, n, X, ld, OUT, ld, p.ncols, static_cast<T>(p.alpha),
                                  static_cast<T>(p.beta), static_cast<T>(p.gamma), ps, stream);
      }
      if (err != hipSuccess) {
        status = err;
        return;
      }
      matvecs += p.ncols;
    });
  }
  if (status != hipSuccess) return status;
  if (matvecs_out) *matvecs_out = matvecs;
  return hipSuccess;
}

template hipError_t run_filter<double>(const double*, int64_t, int64_t, double*, double*, int64_t,
                                       int64_t, const int32_t*, double, double, double,
                                       const ProductScratch&, hipStream_t, int64_t*, int);
template hipError_t run_filter<float>(const float*, int64_t, int64_t, float*, float*, int64_t,
                                      int64_t, const int32_t*, double, double, double,
                                      const ProductScratch&, hipStream_t, int64_t*, int);

}  // namespace chase
