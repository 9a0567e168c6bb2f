// Host side of the Chebyshev filter (Algorithm 4 with the scaled recurrence of Eq. (7)).
//
// The coefficients are scalars computed here in FP64 and passed to each launch:
//   product 1:   W <- (sigma_1/e) (H - cI) V                      (Alg. 4 line 4)
//   product i>1: V[:, s:] <- (2 tau/e)(H - cI) W[:, s:] - tau sigma V[:, s:], swap V, W   (lines 8-10)
// with sigma_1 = e/(mu_1 - c), tau = 1/(2/sigma_1 - sigma) and sigma <- tau.  The active range
// starts at s, the first column whose degree exceeds the products done so far (lines 12-14);
// degrees are sorted, so the range is a contiguous suffix and one launch covers it.

#include "internal.h"

namespace chase {

std::vector<FilterProduct> filter_schedule(int64_t ncols, const int32_t* degrees, double b_sup,
                                           double mu_1, double mu_nevnex) {
  std::vector<FilterProduct> out;
  if (ncols <= 0) return out;
  const double c = 0.5 * (b_sup + mu_nevnex);
  const double e = 0.5 * (b_sup - mu_nevnex);
  const double sigma1 = e / (mu_1 - c);
  const int32_t m_max = degrees[ncols - 1];
  // product 1, every column: W <- a1 H V + g1 V
  double alpha = sigma1 / e;
  out.push_back({/*from_v=*/true, 0, ncols, alpha, 0.0, -alpha * c});
  bool in_is_w = true;  // p_{i-1} lives in W, p_{i-2} in V
  double sigma = sigma1;
  int64_t s = 0;
  while (s < ncols && degrees[s] <= 1) ++s;
  for (int32_t i = 2; i <= m_max; ++i) {
    const double tau = 1.0 / (2.0 / sigma1 - sigma);
    alpha = 2.0 * tau / e;
    out.push_back({/*from_v=*/!in_is_w, s, ncols - s, alpha, -tau * sigma, -alpha * c});
    in_is_w = !in_is_w;
    sigma = tau;
    while (s < ncols && degrees[s] <= i) ++s;
  }
  // m_max is even, so the last product wrote V.
  return out;
}

template <typename T>
hipError_t run_filter(const T* H, int64_t ldh, int64_t n, T* V, T* W, int64_t ld, int64_t ncols,
                      const int32_t* degrees, double b_sup, double mu_1, double mu_nevnex,
                      const ProductScratch& ps, hipStream_t stream, int64_t* matvecs_out) {
  int64_t matvecs = 0;
  if (ncols > 0 && n > 0) {
    for (const FilterProduct& p : filter_schedule(ncols, degrees, b_sup, mu_1, mu_nevnex)) {
      const T* X = (p.from_v ? V : W) + 2 * p.col0 * ld;
      T* OUT = (p.from_v ? W : V) + 2 * p.col0 * ld;
      hipError_t err = launch_hemm_step<T>(H, ldh, n, X, ld, OUT, ld, p.ncols,
                                           static_cast<T>(p.alpha), static_cast<T>(p.beta),
                                           static_cast<T>(p.gamma), ps, stream);
      if (err != hipSuccess) return err;
      matvecs += p.ncols;
    }
  }
  if (matvecs_out) *matvecs_out = matvecs;
  return hipSuccess;
}

template hipError_t run_filter<double>(const double*, int64_t, int64_t, double*, double*, int64_t,
                                       int64_t, const int32_t*, double, double, double,
                                       const ProductScratch&, hipStream_t, int64_t*);
template hipError_t run_filter<float>(const float*, int64_t, int64_t, float*, float*, int64_t,
                                      int64_t, const int32_t*, double, double, double,
                                      const ProductScratch&, hipStream_t, int64_t*);

}  // namespace chase
