// The device-resident outer loop of ChASE (Algorithm 1) and the sequence driver (Sec. 3.3).
//
// Per iteration, all block data stay in device memory:
//   FILTER            Alg. 4 on the active columns, FP64 or (mixed mode) FP32 per column group
//   ORTHOGONALIZE     Alg. 1: block Gram-Schmidt against the locked vectors, column
//                     scaling, shifted Cholesky QR + two Cholesky QR passes; Householder QR of
//                     [Y V] (rocSOLVER) if a Cholesky factorisation breaks down
//   RAYLEIGH-RITZ     Alg. 2: H Q with the filter's product kernel, G = Q^H (H Q) (rocBLAS, K
//                     split into slices so that the tall-skinny product fills the GPU),
//                     TSOLVE = rocSOLVER zheevd, V = Q Z, H V = (H Q) Z
//   residuals         Alg. 1, one fused kernel, then Ritz values and residual norms go to
//                     the host (the only per-iteration device-to-host transfer of results)
//   host              Alg. 3 (locking), Alg. 1 (interval), Alg. 5 (degrees), Alg. 1
//                     (sort); the new column order is applied on the device by one gather.
// LANCZOS (Alg. 6) runs first: the b_sup run and the n_vec DoS runs are independent, so they
// advance together as one block product per step.
// The same loop serves complex Hermitian H (Z routines) and real symmetric H (D routines, real
// product kernel), w_ = values per element (2 or 1), in double precision (R = double) or wholly in
// single precision (R = float: complex64 / float32 data, C and S routines).

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include <rocsolver/rocsolver.h>

#include "host_logic.h"
#include "internal.h"

#include <chrono>
#include <cstdio>

namespace chase {
namespace {

struct Layout {
  size_t V, W, AQ, X, G, T, P, lam, res, evE, perm, info, U, Wl, lal, lbe, zero, Z, tau, H32, V32,
      W32, H64;
  size_t total;
};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// planar64: the planar complex128 copy of H for the FP64 3M products (16 n^2 bytes)
Layout make_layout(int64_t n, int64_t nb, int64_t nv, int64_t k, bool mixed, int w, int esz,
                   bool planar64) {
  Layout L{};
  const size_t es = static_cast<size_t>(esz) * w;  // bytes per element (esz: bytes per scalar)
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t blk = static_cast<size_t>(n) * nb * es;
  L.V = take(blk);
  L.W = take(blk);
  L.AQ = take(blk);
  L.X = take(blk);
  L.G = take(static_cast<size_t>(nb) * nb * es);
  L.T = take(static_cast<size_t>(nb) * nb * es);
  L.P = take(static_cast<size_t>(gram_buffer_elems(nb)) * es);  // K-slices of Gram products
  L.lam = take(nb * 8);
  L.res = take(nb * 8);
  L.evE = take(nb * 8);
  L.perm = take(nb * 4);
  L.info = take(64);
  L.U = take(static_cast<size_t>(n) * nv * (k + 1) * es);
  L.Wl = take(static_cast<size_t>(n) * nv * es);
  L.lal = take(static_cast<size_t>(nv) * k * 8);
  L.lbe = take(static_cast<size_t>(nv) * k * 8);
  L.zero = take(static_cast<size_t>(nv) * 8);
  L.Z = take(static_cast<size_t>(k) * nb * es);
  L.tau = take(nb * 16);
  // FP32 copy of H: planar complex64 (mixed complex, and single-precision complex for the 3M
  // product) or real float32 (mixed real); mixed mode also holds two FP32 blocks
  if (mixed || (esz == 4 && w == 2)) L.H32 = take(static_cast<size_t>(n) * n * 4 * w);
  if (mixed) {
    L.V32 = take(static_cast<size_t>(n) * nb * 4 * w);
    L.W32 = take(static_cast<size_t>(n) * nb * 4 * w);
  }
  if (planar64) L.H64 = take(static_cast<size_t>(n) * n * 16);
  L.total = off;
  return L;
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

template <typename R>  // device scalar: double (complex128 / float64) or float (complex64 / float32)
class Solver {
 public:
  Solver(chase_ctx* ctx, const chase_config& cfg, Batcher* batcher)
      : ctx_(ctx), cfg_(cfg), batcher_(batcher) {}
  int run(const void* H, int64_t ldh, void* Vuser, int64_t ldv, double* ritzv, double* resid,
          chase_stats* stats);

 private:
  chase_ctx* ctx_;
  chase_config cfg_;
  Batcher* batcher_ = nullptr;
  hipEvent_t bev_[2] = {nullptr, nullptr};  // events handed to the batcher (ready, done)
  Layout L_{};
  char* base_ = nullptr;
  int64_t n_ = 0, nb_ = 0;
  int w_ = 2;             // values per element: 2 complex, 1 real
  bool real_ = false;
  bool planar64_ = false;  // FP64 3M products on the planar copy of H at L_.H64
  hipStream_t s_ = nullptr;
  chase_stats st_{};
  int fallbacks_ = 0;

  template <typename P> P* at(size_t off) { return reinterpret_cast<P*>(base_ + off); }
  R* col(size_t off, int64_t c) { return at<R>(off) + w_ * c * n_; }
  size_t es() const { return sizeof(R) * static_cast<size_t>(w_); }
  static constexpr bool kF64 = sizeof(R) == 8;
  // unit roundoff of R
  static constexpr double kU = kF64 ? 1.1102230246251565e-16 : 5.9604644775390625e-08;

  int blas(rocblas_status s, const char* what) {
    if (s != rocblas_status_success)
      return set_error(ctx_, CHASE_EDEVICE, std::string(what) + ": rocBLAS/rocSOLVER status " +
                                                std::to_string(static_cast<int>(s)));
    return CHASE_OK;
  }
  int hip(hipError_t e, const char* what) {
    if (e != hipSuccess)
      return set_error(ctx_, CHASE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return CHASE_OK;
  }
  // C <- ar op(A) op(B) + br C with real scalars; conjugate transpose is the transpose for real
  // data.
  int gemm(rocblas_operation ta, rocblas_operation tb, int64_t m, int64_t nn, int64_t k,
           double ar, const R* A, int64_t lda, const R* B, int64_t ldb, double br, R* C,
           int64_t ldc) {
    const rocblas_int im = static_cast<rocblas_int>(m), in = static_cast<rocblas_int>(nn),
                      ik = static_cast<rocblas_int>(k), ia = static_cast<rocblas_int>(lda),
                      ib = static_cast<rocblas_int>(ldb), ic = static_cast<rocblas_int>(ldc);
    if (real_) {
      auto rt = [](rocblas_operation o) {
        return o == rocblas_operation_conjugate_transpose ? rocblas_operation_transpose : o;
      };
      if constexpr (kF64) {
        return blas(rocblas_dgemm(ctx_->blas, rt(ta), rt(tb), im, in, ik, &ar, A, ia, B, ib, &br,
                                  C, ic),
                    "dgemm");
      } else {
        const float af = static_cast<float>(ar), bf = static_cast<float>(br);
        return blas(rocblas_sgemm(ctx_->blas, rt(ta), rt(tb), im, in, ik, &af, A, ia, B, ib, &bf,
                                  C, ic),
                    "sgemm");
      }
    }
    if constexpr (!kF64) {
      const rocblas_float_complex al(static_cast<float>(ar), 0.f), be(static_cast<float>(br), 0.f);
      return blas(rocblas_cgemm(ctx_->blas, ta, tb, im, in, ik, &al,
                                reinterpret_cast<const rocblas_float_complex*>(A), ia,
                                reinterpret_cast<const rocblas_float_complex*>(B), ib, &be,
                                reinterpret_cast<rocblas_float_complex*>(C), ic),
                  "cgemm");
    } else {
      const rocblas_double_complex al(ar, 0.0), be(br, 0.0);
      return blas(rocblas_zgemm(ctx_->blas, ta, tb, im, in, ik, &al,
                                reinterpret_cast<const rocblas_double_complex*>(A), ia,
                                reinterpret_cast<const rocblas_double_complex*>(B), ib, &be,
                                reinterpret_cast<rocblas_double_complex*>(C), ic),
                  "zgemm");
    }
  }
  // OUT <- alpha H X + gamma X + beta OUT with the product kernel of the element type.
  // G (ld ldg) <- A^H B for n x m1 A and n x m2 B (ld n): a batch of K-slice products into the
  // slice buffer, then their sum (one GEMM when the result alone fills the GPU).
  int gram(int64_t m1, int64_t m2, const R* A, const R* B, R* G, int64_t ldg) {
    int64_t p = gram_slices(m1, m2, n_);
    const int64_t cap = gram_buffer_elems(nb_);
    if (p * m1 * m2 > cap) p = cap / (m1 * m2);
    const auto ct = rocblas_operation_conjugate_transpose, nn = rocblas_operation_none;
    if (p <= 1) return gemm(ct, nn, m1, m2, n_, 1.0, A, n_, B, n_, 0.0, G, ldg);
    const int64_t kc = n_ / p, rem = n_ - p * kc;
    R* P = at<R>(L_.P);
    int rc = gemm_sb(m1, m2, kc, A, B, P, p);
    if (rc) return rc;
    if (rem > 0 &&
        (rc = gemm(ct, nn, m1, m2, rem, 1.0, A + w_ * p * kc, n_, B + w_ * p * kc, n_, 1.0, P, m1)))
      return rc;
    return hip(launch_sum_slices(P, m1, m2, m1 * m2, static_cast<int>(p), G, ldg, s_, w_),
               "sum slices");
  }
  // Slice q of P (m1 x m2, ld m1) <- A[q kc : (q+1) kc, :]^H B[q kc : (q+1) kc, :], q < p.
  int gemm_sb(int64_t m1, int64_t m2, int64_t kc, const R* A, const R* B, R* P, int64_t p) {
    const rocblas_int im = static_cast<rocblas_int>(m1), in = static_cast<rocblas_int>(m2),
                      ik = static_cast<rocblas_int>(kc), ld = static_cast<rocblas_int>(n_),
                      bc = static_cast<rocblas_int>(p);
    const rocblas_stride sk = kc, sp = m1 * m2;
    const auto nn = rocblas_operation_none;
    if constexpr (kF64) {
      if (real_) {
        const double one = 1.0, zero = 0.0;
        return blas(rocblas_dgemm_strided_batched(ctx_->blas, rocblas_operation_transpose, nn, im,
                                                  in, ik, &one, A, ld, sk, B, ld, sk, &zero, P, im,
                                                  sp, bc),
                    "dgemm batched");
      }
      const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
      return blas(rocblas_zgemm_strided_batched(
                      ctx_->blas, rocblas_operation_conjugate_transpose, nn, im, in, ik, &one,
                      reinterpret_cast<const rocblas_double_complex*>(A), ld, sk,
                      reinterpret_cast<const rocblas_double_complex*>(B), ld, sk, &zero,
                      reinterpret_cast<rocblas_double_complex*>(P), im, sp, bc),
                  "zgemm batched");
    } else {
      if (real_) {
        const float one = 1.f, zero = 0.f;
        return blas(rocblas_sgemm_strided_batched(ctx_->blas, rocblas_operation_transpose, nn, im,
                                                  in, ik, &one, A, ld, sk, B, ld, sk, &zero, P, im,
                                                  sp, bc),
                    "sgemm batched");
      }
      const rocblas_float_complex one(1.f, 0.f), zero(0.f, 0.f);
      return blas(rocblas_cgemm_strided_batched(
                      ctx_->blas, rocblas_operation_conjugate_transpose, nn, im, in, ik, &one,
                      reinterpret_cast<const rocblas_float_complex*>(A), ld, sk,
                      reinterpret_cast<const rocblas_float_complex*>(B), ld, sk, &zero,
                      reinterpret_cast<rocblas_float_complex*>(P), im, sp, bc),
                  "cgemm batched");
    }
  }
  hipError_t product(const R* H, int64_t ldh, const R* X, int64_t ldx, R* OUT, int64_t ldo,
                     int64_t ncols, double alpha, double beta, double gamma) {
    const R a = static_cast<R>(alpha), b = static_cast<R>(beta), g = static_cast<R>(gamma);
    if (real_)
      return launch_hemm_step_real<R>(H, ldh, n_, X, ldx, OUT, ldo, ncols, a, b, g, ctx_->prod, s_);
    if constexpr (kF64) {
      // 3M on the planar copy for wide blocks (Rayleigh-Ritz); thin Lanczos blocks read one
      // triangle of H where that pays and its partial sums fit the product scratch, else 4M
      if (planar64_ && ncols > 16)
        return launch_hemm_step_3m_f64(at<double>(L_.H64), n_, n_, X, ldx, OUT, ldo, ncols, alpha,
                                       beta, gamma, ctx_->prod, s_);
      if (ncols <= kTriSolverCols && n_ >= kTriMinOrder &&
          tri_scratch_bytes(n_, ncols) <= ctx_->prod.bytes)
        return launch_hemm_tri(H, ldh, n_, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, ctx_->prod,
                               s_);
    }
    return launch_hemm_step<R>(H, ldh, n_, X, ldx, OUT, ldo, ncols, a, b, g, ctx_->prod, s_);
  }
  int lanczos(const R* H, int64_t ldh, R* V);
  int cgs(int64_t nlock, int64_t nact);
  int cholqr(int64_t nact, bool shift, int slot);
  int householder(int64_t nlock, int64_t nact);
  int orthogonalize(int64_t nlock, int64_t nact);
  int filter(const R* H, int64_t ldh, int64_t nlock, int64_t nact,
             const std::vector<int>& m, const std::vector<int>& prec);
  int filter_mixed(const R* H, int64_t ldh, int64_t nlock, int64_t nact,
                   const std::vector<int>& m, const std::vector<int>& prec);

  double b_sup_ = 0, mu_1_ = 0, mu_b_ = 0, norm_est_ = 0;
};

template <typename R>
int Solver<R>::lanczos(const R* H, int64_t ldh, R* V) {
  const bool need_dos = !cfg_.approx && !cfg_.have_mu;
  const int64_t nv = need_dos ? 1 + cfg_.num_lanczos : 1;
  const int k = static_cast<int>(std::min<int64_t>(cfg_.lanczos_iter, n_));
  R* U = at<R>(L_.U);
  int rc;
  if (cfg_.lanczos_start) {
    rc = hip(hipMemcpyAsync(U, cfg_.lanczos_start, static_cast<size_t>(n_) * nv * es(),
                            hipMemcpyDeviceToDevice, s_),
             "copy lanczos start");
  } else {
    rc = hip(launch_gaussian(U, n_, n_, nv, cfg_.seed, s_, w_), "gaussian");
  }
  if (rc) return rc;
  if ((rc = hip(launch_normalize(U, n_, n_, nv, s_, w_), "normalize"))) return rc;
  if ((rc = hip(hipMemsetAsync(at<double>(L_.zero), 0, nv * 8, s_), "memset"))) return rc;
  R* Wl = at<R>(L_.Wl);
  for (int j = 0; j < k; ++j) {
    R* Uj = U + w_ * static_cast<int64_t>(j) * nv * n_;
    const R* Up = j > 0 ? U + w_ * static_cast<int64_t>(j - 1) * nv * n_ : Uj;
    const double* bp = j > 0 ? at<double>(L_.lbe) + (j - 1) * nv : at<double>(L_.zero);
    if ((rc = hip(product(H, ldh, Uj, n_, Wl, n_, nv, 1.0, 0.0, 0.0), "lanczos product")))
      return rc;
    if ((rc = hip(launch_lanczos_step(Uj, Up, Wl, Uj + w_ * nv * n_, n_, n_, nv, bp,
                                      at<double>(L_.lal) + j * nv, at<double>(L_.lbe) + j * nv, s_,
                                      w_),
                  "lanczos step")))
      return rc;
  }
  std::vector<double> al(static_cast<size_t>(nv) * k), be(static_cast<size_t>(nv) * k);
  if ((rc = hip(hipMemcpyAsync(al.data(), at<double>(L_.lal), al.size() * 8, hipMemcpyDeviceToHost,
                               s_), "d2h")))
    return rc;
  if ((rc = hip(hipMemcpyAsync(be.data(), at<double>(L_.lbe), be.size() * 8, hipMemcpyDeviceToHost,
                               s_), "d2h")))
    return rc;
  if ((rc = hip(hipStreamSynchronize(s_), "sync"))) return rc;
  st_.matvecs += static_cast<int64_t>(k) * nv;
  for (double x : al)
    if (!std::isfinite(x)) return set_error(ctx_, CHASE_ENUMERIC, "Lanczos produced NaN/Inf");

  LanczosRun r0 = tridiag_eig(al, be, static_cast<int>(nv), 0, k);
  b_sup_ = r0.beta_last + r0.ritz.back();                      // Alg. 6 upper bound
  norm_est_ = std::max(std::fabs(r0.ritz.front()), std::fabs(r0.ritz.back()));
  if (!need_dos) return CHASE_OK;

  std::vector<LanczosRun> runs;
  double lo = INFINITY;
  for (int c = 1; c < nv; ++c) {
    runs.push_back(tridiag_eig(al, be, static_cast<int>(nv), c, k));
    lo = std::min(lo, runs.back().ritz.front());
  }
  mu_1_ = lo;                                                   // Alg. 6 DoS estimate
  mu_b_ = dos_mu(runs, lo, b_sup_, cfg_.dos_sigma,
                 static_cast<double>(nb_) / static_cast<double>(n_));
  if (cfg_.intersperse) {                                       // Alg. 6 returned vectors
    const LanczosRun& r1 = runs.front();
    std::vector<int> sel;
    for (int i = 0; i < r1.k; ++i)
      if (r1.ritz[i] < mu_b_) sel.push_back(i);
    if (static_cast<int64_t>(sel.size()) > nb_) sel.resize(nb_);
    const int64_t r = static_cast<int64_t>(sel.size());
    if (r > 0) {
      std::vector<R> Zh(static_cast<size_t>(r1.k) * r * w_, R(0));  // k x r, col-major
      for (int64_t q = 0; q < r; ++q)
        for (int j = 0; j < r1.k; ++j)
          Zh[w_ * (j + q * r1.k)] = static_cast<R>(r1.evecs[j * r1.k + sel[q]]);
      if ((rc = hip(hipMemcpyAsync(at<R>(L_.Z), Zh.data(), Zh.size() * sizeof(R),
                                   hipMemcpyHostToDevice, s_), "h2d")))
        return rc;
      // basis of DoS run 1: columns U_j[:, 1], j < k, stride nv*n between consecutive j
      if ((rc = gemm(rocblas_operation_none, rocblas_operation_none, n_, r, r1.k, 1.0,
                      U + w_ * n_, nv * n_, at<R>(L_.Z), r1.k, 0.0, V, n_)))
        return rc;
      if ((rc = hip(hipStreamSynchronize(s_), "sync"))) return rc;
    }
  }
  return CHASE_OK;
}

// Block classical Gram-Schmidt of the active block against the locked prefix Y = V[:, :nlock].
template <typename R>
int Solver<R>::cgs(int64_t nlock, int64_t nact) {
  if (nlock == 0) return CHASE_OK;
  R* Y = at<R>(L_.V);
  R* A = col(L_.V, nlock);
  R* T = at<R>(L_.T);
  int rc = gram(nlock, nact, Y, A, T, nb_);
  if (rc) return rc;
  return gemm(rocblas_operation_none, rocblas_operation_none, n_, nact, nlock, -1.0, Y, n_, T, nb_,
               1.0, A, n_);
}

// One (optionally shifted) Cholesky QR pass on the active block: G = A^H A (+ s I) = R^H R,
// A <- A R^-1.  Shift as in shifted CholeskyQR3 (Fukaya et al.), 11 (n m + m (m + 1)) u ||A||^2
// with ||A||_2^2 <= m = nact for unit columns, capped at 1e-2 m.  The cap only acts in single
// precision at large n (at n = 1e4, m = 600 the FP32 bound is about 4 m): a shift above
// ||A||_2^2 would make the pass a mere rescaling of the block, while 1e-2 m still exceeds the
// Gram matrix's rounding error (about sqrt(n) u m) and bounds the pass's output condition
// number by about sqrt(1e-2 m) / sigma_min(A).
template <typename R>
int Solver<R>::cholqr(int64_t nact, bool shift, int slot) {
  R* A = col(L_.V, n_ == 0 ? 0 : (nb_ - nact));
  R* G = at<R>(L_.G);
  // Gram matrix by K-sliced GEMM (both triangles; faster than HERK at these shapes)
  int rc = gram(nact, nact, A, A, G, nb_);
  if (rc) return rc;
  if (shift) {
    const double m = static_cast<double>(nact);
    const double s =
        std::min(11.0 * (static_cast<double>(n_) * m + m * (m + 1.0)) * kU * m, 1e-2 * m);
    if ((rc = hip(launch_add_diag(G, nb_, nact, s, s_, w_), "add_diag"))) return rc;
  }
  rocblas_int* info = at<rocblas_int>(L_.info) + slot;
  const rocblas_int ia = static_cast<rocblas_int>(nact), ig = static_cast<rocblas_int>(nb_),
                    in = static_cast<rocblas_int>(n_);
  // own factorisation: its summation order is fixed, so the factor does not depend on what
  // else runs on the device
  rc = hip(launch_potrf_upper(G, nb_, nact, info, s_, w_), "potrf");
  if (rc) return rc;
  // The factorisation status is read once per orthonormalisation (see orthogonalize); a failed
  // factorisation makes this solve produce garbage that is then discarded.
  if constexpr (!kF64) {
    const float one = 1.f;
    const rocblas_float_complex al(1.f, 0.f);
    if (real_)
      return blas(rocblas_strsm(ctx_->blas, rocblas_side_right, rocblas_fill_upper,
                                rocblas_operation_none, rocblas_diagonal_non_unit, in, ia, &one, G,
                                ig, A, in),
                  "strsm");
    return blas(rocblas_ctrsm(ctx_->blas, rocblas_side_right, rocblas_fill_upper,
                              rocblas_operation_none, rocblas_diagonal_non_unit, in, ia, &al,
                              reinterpret_cast<const rocblas_float_complex*>(G), ig,
                              reinterpret_cast<rocblas_float_complex*>(A), in),
                "ctrsm");
  } else {
    const double one = 1.0;
    const rocblas_double_complex al(1.0, 0.0);
    if (real_)
      return blas(rocblas_dtrsm(ctx_->blas, rocblas_side_right, rocblas_fill_upper,
                                rocblas_operation_none, rocblas_diagonal_non_unit, in, ia, &one, G,
                                ig, A, in),
                  "dtrsm");
    return blas(rocblas_ztrsm(ctx_->blas, rocblas_side_right, rocblas_fill_upper,
                              rocblas_operation_none, rocblas_diagonal_non_unit, in, ia, &al,
                              reinterpret_cast<const rocblas_double_complex*>(G), ig,
                              reinterpret_cast<rocblas_double_complex*>(A), in),
                "ztrsm");
  }
}

// Householder QR of [Y V] (the paper's ORTHOGONALIZE), keeping the columns after Y.
template <typename R>
int Solver<R>::householder(int64_t nlock, int64_t nact) {
  ++fallbacks_;
  const int64_t ncol = nlock + nact;
  R* Wb = at<R>(L_.W);
  int rc = hip(hipMemcpyAsync(Wb, at<R>(L_.V), static_cast<size_t>(n_) * ncol * es(),
                              hipMemcpyDeviceToDevice, s_),
               "copy");
  if (rc) return rc;
  const rocblas_int in = static_cast<rocblas_int>(n_), ic = static_cast<rocblas_int>(ncol);
  if constexpr (kF64) {
    if (real_) {
      double* tau = at<double>(L_.tau);
      if ((rc = blas(rocsolver_dgeqrf(ctx_->blas, in, ic, Wb, in, tau), "dgeqrf"))) return rc;
      if ((rc = blas(rocsolver_dorgqr(ctx_->blas, in, ic, ic, Wb, in, tau), "dorgqr"))) return rc;
    } else {
      auto* Wz = reinterpret_cast<rocblas_double_complex*>(Wb);
      auto* tau = at<rocblas_double_complex>(L_.tau);
      if ((rc = blas(rocsolver_zgeqrf(ctx_->blas, in, ic, Wz, in, tau), "zgeqrf"))) return rc;
      if ((rc = blas(rocsolver_zungqr(ctx_->blas, in, ic, ic, Wz, in, tau), "zungqr"))) return rc;
    }
  } else {
    if (real_) {
      float* tau = at<float>(L_.tau);
      if ((rc = blas(rocsolver_sgeqrf(ctx_->blas, in, ic, Wb, in, tau), "sgeqrf"))) return rc;
      if ((rc = blas(rocsolver_sorgqr(ctx_->blas, in, ic, ic, Wb, in, tau), "sorgqr"))) return rc;
    } else {
      auto* Wc = reinterpret_cast<rocblas_float_complex*>(Wb);
      auto* tau = at<rocblas_float_complex>(L_.tau);
      if ((rc = blas(rocsolver_cgeqrf(ctx_->blas, in, ic, Wc, in, tau), "cgeqrf"))) return rc;
      if ((rc = blas(rocsolver_cungqr(ctx_->blas, in, ic, ic, Wc, in, tau), "cungqr"))) return rc;
    }
  }
  return hip(hipMemcpyAsync(col(L_.V, nlock), Wb + w_ * nlock * n_,
                            static_cast<size_t>(n_) * nact * es(), hipMemcpyDeviceToDevice, s_),
             "copy");
}

// The three Cholesky factorisations report their status into three slots that are read with
// one synchronisation at the end; if any failed, the filtered block is restored from its copy in
// W and orthonormalised by Householder QR instead.
template <typename R>
int Solver<R>::orthogonalize(int64_t nlock, int64_t nact) {
  int rc;
  R* A = col(L_.V, nlock);
  R* B = col(L_.W, nlock);  // W is free between the filter and Rayleigh-Ritz
  if ((rc = hip(hipMemcpyAsync(B, A, static_cast<size_t>(n_) * nact * es(),
                               hipMemcpyDeviceToDevice, s_), "copy")))
    return rc;
  if ((rc = cgs(nlock, nact))) return rc;
  if ((rc = hip(launch_normalize(A, n_, n_, nact, s_, w_), "normalize"))) return rc;
  if ((rc = cholqr(nact, true, 0))) return rc;
  if ((rc = cgs(nlock, nact))) return rc;
  if ((rc = cholqr(nact, false, 1))) return rc;
  if ((rc = cholqr(nact, false, 2))) return rc;
  int info[3] = {0, 0, 0};
  if ((rc = hip(hipMemcpyAsync(info, at<int>(L_.info), sizeof(info), hipMemcpyDeviceToHost, s_),
                "info")))
    return rc;
  if ((rc = hip(hipStreamSynchronize(s_), "sync"))) return rc;
  if (info[0] == 0 && info[1] == 0 && info[2] == 0) return CHASE_OK;
  if ((rc = hip(hipMemcpyAsync(A, B, static_cast<size_t>(n_) * nact * es(),
                               hipMemcpyDeviceToDevice, s_), "copy")))
    return rc;
  return householder(nlock, nact);
}

template <typename R>
int Solver<R>::filter(const R* H, int64_t ldh, int64_t nlock, int64_t nact,
                      const std::vector<int>& m, const std::vector<int>& prec) {
  if constexpr (!kF64) {  // single-precision solve: 3M on the planar copy of H, or real FP32
    int64_t mv = 0;
    const int rc =
        real_ ? hip(run_filter<float>(H, ldh, n_, col(L_.V, nlock), col(L_.W, nlock), n_, nact,
                                      m.data(), b_sup_, mu_1_, mu_b_, ctx_->prod, s_, &mv, 3),
                    "filter real fp32")
              : hip(run_filter<float>(at<float>(L_.H32), n_, n_, col(L_.V, nlock),
                                      col(L_.W, nlock), n_, nact, m.data(), b_sup_, mu_1_, mu_b_,
                                      ctx_->prod, s_, &mv, 2),
                    "filter fp32 3M");
    if (rc) return rc;
    st_.filter_matvecs += mv;
    return CHASE_OK;
  } else {
    return filter_mixed(H, ldh, nlock, nact, m, prec);
  }
}

// Double-precision data: the FP32 column group first (mixed mode), then the FP64 group.
template <typename R>
int Solver<R>::filter_mixed(const R* H, int64_t ldh, int64_t nlock, int64_t nact,
                            const std::vector<int>& m, const std::vector<int>& prec) {
  int64_t n32 = 0;
  while (n32 < nact && prec[n32] == 1) ++n32;
  int rc;
  int64_t mv = 0;
  if (n32 > 0) {
    float* V32 = at<float>(L_.V32);
    if (real_) {  // real float32 filter on the float32 copy of H
      if ((rc = hip(launch_convert_f64_to_f32(col(L_.V, nlock), n_, V32, n_, n_, n32, s_), "cvt")))
        return rc;
      if ((rc = hip(run_filter<float>(at<float>(L_.H32), n_, n_, V32, at<float>(L_.W32), n_, n32,
                                      m.data(), b_sup_, mu_1_, mu_b_, ctx_->prod, s_, &mv, 3),
                    "filter real fp32")))
        return rc;
      st_.filter_matvecs += mv;
      if ((rc = hip(launch_convert_f32_to_f64(V32, n_, col(L_.V, nlock), n_, n_, n32, s_), "cvt")))
        return rc;
    }
  }
  if (n32 > 0 && !real_) {
    float* V32 = at<float>(L_.V32);
    if ((rc = hip(launch_convert_c128_to_c64(col(L_.V, nlock), n_, V32, n_, n_, n32, s_), "cvt")))
      return rc;
    if (batcher_) {
      const auto prods = filter_schedule(n32, m.data(), b_sup_, mu_1_, mu_b_);
      mv = 0;
      for (const auto& p : prods) mv += p.ncols;
      rc = hip(batcher_->run(2, at<float>(L_.H32), n_, n_, V32, at<float>(L_.W32), n_, prods,
                             s_, bev_[0], bev_[1]),
               "batched filter fp32");
    } else {
      rc = hip(run_filter<float>(at<float>(L_.H32), n_, n_, V32, at<float>(L_.W32), n_, n32,
                                 m.data(), b_sup_, mu_1_, mu_b_, ctx_->prod, s_, &mv, 2),
               "filter fp32");
    }
    if (rc) return rc;
    st_.filter_matvecs += mv;
    if ((rc = hip(launch_convert_c64_to_c128(V32, n_, col(L_.V, nlock), n_, n_, n32, s_), "cvt")))
      return rc;
  }
  if (nact - n32 > 0 && real_) {
    if ((rc = hip(run_filter<double>(H, ldh, n_, col(L_.V, nlock + n32), col(L_.W, nlock + n32), n_,
                                     nact - n32, m.data() + n32, b_sup_, mu_1_, mu_b_, ctx_->prod,
                                     s_, &mv, 3),
                  "filter real fp64")))
      return rc;
    st_.filter_matvecs += mv;
  } else if (nact - n32 > 0) {
    if (batcher_) {
      const auto prods = filter_schedule(nact - n32, m.data() + n32, b_sup_, mu_1_, mu_b_);
      mv = 0;
      for (const auto& p : prods) mv += p.ncols;
      rc = planar64_
               ? hip(batcher_->run(3, at<double>(L_.H64), n_, n_, col(L_.V, nlock + n32),
                                   col(L_.W, nlock + n32), n_, prods, s_, bev_[0], bev_[1]),
                     "batched filter fp64 3M")
               : hip(batcher_->run(0, H, ldh, n_, col(L_.V, nlock + n32), col(L_.W, nlock + n32),
                                   n_, prods, s_, bev_[0], bev_[1]),
                     "batched filter fp64");
    } else if (planar64_) {  // 3M on the planar copy of H
      rc = hip(run_filter<double>(at<double>(L_.H64), n_, n_, col(L_.V, nlock + n32),
                                  col(L_.W, nlock + n32), n_, nact - n32, m.data() + n32, b_sup_,
                                  mu_1_, mu_b_, ctx_->prod, s_, &mv, 4),
               "filter fp64 3M");
    } else {
      rc = hip(run_filter<double>(H, ldh, n_, col(L_.V, nlock + n32), col(L_.W, nlock + n32), n_,
                                  nact - n32, m.data() + n32, b_sup_, mu_1_, mu_b_, ctx_->prod, s_,
                                  &mv),
               "filter fp64");
    }
    if (rc) return rc;
    st_.filter_matvecs += mv;
  }
  return CHASE_OK;
}

template <typename R>
int Solver<R>::run(const void* Hv, int64_t ldh, void* Vuser, int64_t ldv, double* ritzv, double* resid,
                chase_stats* stats) {
  const R* H = static_cast<const R*>(Hv);
  n_ = cfg_.n;
  nb_ = cfg_.nev + cfg_.nex;
  real_ = cfg_.real_symmetric != 0;
  w_ = real_ ? 1 : 2;
  planar64_ = kF64 && !real_ && cfg_.filter_3m != 0;
  s_ = ctx_->stream;
  const bool mixed = cfg_.precision == CHASE_MIXED;
  const bool need_dos = !cfg_.approx && !cfg_.have_mu;
  const int64_t nv = need_dos ? 1 + cfg_.num_lanczos : 1;
  const int64_t k = std::min<int64_t>(cfg_.lanczos_iter, n_);
  L_ = make_layout(n_, nb_, nv, k, mixed, w_, static_cast<int>(sizeof(R)), planar64_);
  int rc = ensure_workspace(ctx_, L_.total);
  if (rc) return rc;
  base_ = static_cast<char*>(ctx_->ws);
  std::memset(&st_, 0, sizeof(st_));

  hipEvent_t ev[8];
  for (auto& e : ev)
    if ((rc = hip(hipEventCreate(&e), "event"))) return rc;
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 8; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  struct BevGuard {
    hipEvent_t* e;
    hipStream_t s;
    ~BevGuard() {
      if (e[0] || e[1]) (void)hipStreamSynchronize(s);
      for (int i = 0; i < 2; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } bguard{bev_, s_};
  if (batcher_)
    for (auto& e : bev_)
      if ((rc = hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event"))) return rc;
  auto elapsed = [&](int a, int b) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
    return static_cast<double>(ms);
  };

  (void)hipEventRecord(ev[6], s_);
  // state: V (ld n) <- user block
  if ((rc = hip(hipMemcpy2DAsync(at<R>(L_.V), n_ * es(), Vuser, ldv * es(), n_ * es(), nb_,
                                 hipMemcpyDeviceToDevice, s_),
                "copy V")))
    return rc;
  if constexpr (!kF64) {
    if (!real_ &&
        (rc = hip(launch_split_planes_c64(H, ldh, at<float>(L_.H32), n_, n_, s_), "planar H")))
      return rc;
  }
  if constexpr (kF64) {
    if (planar64_ &&
        (rc = hip(launch_convert_c128_to_planar64(H, ldh, at<double>(L_.H64), n_, n_, s_),
                  "planar H")))
      return rc;
    if (mixed && real_ &&
        (rc = hip(launch_convert_f64_to_f32(H, ldh, at<float>(L_.H32), n_, n_, n_, s_),
                  "convert H")))
      return rc;
    if (mixed && !real_ &&
        (rc = hip(launch_convert_c128_to_planar32(H, ldh, at<float>(L_.H32), n_, n_, s_),
                  "convert H")))
      return rc;
  }

  // ---------------------------------------------------------------- LANCZOS (Alg. 1, Alg. 6)
  (void)hipEventRecord(ev[0], s_);
  if ((rc = lanczos(H, ldh, at<R>(L_.V)))) return rc;
  (void)hipEventRecord(ev[1], s_);
  if (cfg_.approx) {
    double lo = ritzv[0], hi = ritzv[0];
    for (int64_t i = 1; i < nb_; ++i) {
      lo = std::min(lo, ritzv[i]);
      hi = std::max(hi, ritzv[i]);
    }
    mu_1_ = lo;
    mu_b_ = hi;
  } else if (cfg_.have_mu) {
    mu_1_ = cfg_.mu_1;
    mu_b_ = cfg_.mu_nevnex;
  }
  if (!(mu_1_ < mu_b_ && mu_b_ < b_sup_)) {
    // degenerate bounds (e.g. a warm start whose Ritz values all coincide): widen minimally
    if (!(mu_b_ < b_sup_)) mu_b_ = 0.5 * (mu_1_ + b_sup_);
    if (!(mu_1_ < mu_b_)) mu_1_ = mu_b_ - 1e-3 * (b_sup_ - mu_b_);
  }
  (void)hipEventSynchronize(ev[1]);
  st_.lanczos_ms = elapsed(0, 1);
  const double tol_eff = cfg_.resid_relative ? cfg_.tol * norm_est_ : cfg_.tol;
  const double tol32 = cfg_.resid_relative ? cfg_.switch_resid * norm_est_ : cfg_.switch_resid;
  const int deg0 = cfg_.deg + (cfg_.deg & 1);
  const int deg32max = cfg_.deg_max_fp32 + (cfg_.deg_max_fp32 & 1);

  // ---------------------------------------------------------------- main loop (Alg. 1)
  const auto t_start = std::chrono::steady_clock::now();
  int64_t nlock = 0;
  std::vector<int> m(nb_, mixed ? std::min(deg0, deg32max) : deg0);
  std::vector<int> prec(nb_, mixed ? 1 : 0);
  // Mixed mode history, indexed by ascending Ritz rank among the active pairs: last residual,
  // whether that pair was filtered in FP32, and a sticky FP64 flag set when an FP32 iteration
  // failed to halve the residual (the FP32 filter's accuracy floor was reached).
  std::vector<double> hist_res(nb_, INFINITY);
  std::vector<char> hist_fp32(nb_, mixed ? 1 : 0), lock64(nb_, 0);
  std::vector<double> lam_act(nb_, 0.0), res_act(nb_, 0.0), lam_lock, res_lock;
  std::vector<R> lam_dev(nb_);
  std::vector<int> perm(nb_);
  int it = 0;
  while (nlock < cfg_.nev && it < cfg_.max_iter) {
    ++it;
    const int64_t nact = nb_ - nlock;
    bool any32 = false;
    for (int64_t a = 0; a < nact; ++a) any32 |= prec[a] == 1;
    if (any32) ++st_.fp32_iterations;
    (void)hipEventRecord(ev[0], s_);
    if ((rc = filter(H, ldh, nlock, nact, m, prec))) return rc;             // FILTER
    (void)hipEventRecord(ev[1], s_);
    if ((rc = orthogonalize(nlock, nact))) return rc;                       // ORTHOGONALIZE
    (void)hipEventRecord(ev[2], s_);
    // RAYLEIGH-RITZ (Alg. 2)
    R* Q = col(L_.V, nlock);
    R* AQ = at<R>(L_.AQ);
    R* G = at<R>(L_.G);
    if ((rc = hip(product(H, ldh, Q, n_, AQ, n_, nact, 1.0, 0.0, 0.0), "H Q"))) return rc;
    st_.matvecs += nact;
    if ((rc = gram(nact, nact, Q, AQ, G, nb_))) return rc;
    if ((rc = hip(launch_herm_sym(G, nb_, nact, s_, w_), "sym"))) return rc;
    {
      const rocblas_int ia = static_cast<rocblas_int>(nact), ig = static_cast<rocblas_int>(nb_);
      R* lam = at<R>(L_.lam);
      R* evE = at<R>(L_.evE);
      rocblas_int* inf = at<rocblas_int>(L_.info);
      const auto ev = rocblas_evect_original;
      const auto up = rocblas_fill_upper;
      if constexpr (kF64)
        rc = real_ ? blas(rocsolver_dsyevd(ctx_->blas, ev, up, ia, G, ig, lam, evE, inf), "dsyevd")
                   : blas(rocsolver_zheevd(ctx_->blas, ev, up, ia,
                                           reinterpret_cast<rocblas_double_complex*>(G), ig, lam,
                                           evE, inf),
                          "zheevd");
      else
        rc = real_ ? blas(rocsolver_ssyevd(ctx_->blas, ev, up, ia, G, ig, lam, evE, inf), "ssyevd")
                   : blas(rocsolver_cheevd(ctx_->blas, ev, up, ia,
                                           reinterpret_cast<rocblas_float_complex*>(G), ig, lam,
                                           evE, inf),
                          "cheevd");
    }
    if (rc) return rc;
    R* Wb = at<R>(L_.W);
    R* Xb = at<R>(L_.X);
    if ((rc = gemm(rocblas_operation_none, rocblas_operation_none, n_, nact, nact, 1.0, Q, n_, G,
                    nb_, 0.0, Wb, n_)))
      return rc;
    if ((rc = gemm(rocblas_operation_none, rocblas_operation_none, n_, nact, nact, 1.0, AQ, n_, G,
                    nb_, 0.0, Xb, n_)))
      return rc;
    (void)hipEventRecord(ev[3], s_);
    // residuals
    if ((rc = hip(launch_resid(Xb, Wb, at<R>(L_.lam), n_, n_, nact, at<double>(L_.res), s_,
                               w_),
                  "resid")))
      return rc;
    if ((rc = hip(hipMemcpyAsync(Q, Wb, static_cast<size_t>(n_) * nact * es(),
                                 hipMemcpyDeviceToDevice, s_),
                  "copy")))
      return rc;
    int info = 0;
    if ((rc = hip(hipMemcpyAsync(lam_dev.data(), at<R>(L_.lam), nact * sizeof(R),
                                 hipMemcpyDeviceToHost, s_), "d2h")))
      return rc;
    if ((rc = hip(hipMemcpyAsync(res_act.data(), at<double>(L_.res), nact * 8,
                                 hipMemcpyDeviceToHost, s_), "d2h")))
      return rc;
    if ((rc = hip(hipMemcpyAsync(&info, at<int>(L_.info), sizeof(int), hipMemcpyDeviceToHost, s_),
                  "d2h")))
      return rc;
    (void)hipEventRecord(ev[4], s_);
    if ((rc = hip(hipStreamSynchronize(s_), "sync"))) return rc;
    st_.filter_ms += elapsed(0, 1);
    st_.ortho_ms += elapsed(1, 2);
    st_.rr_ms += elapsed(2, 3);
    st_.resid_ms += elapsed(3, 4);
    if (info != 0) return set_error(ctx_, CHASE_ENUMERIC, "Rayleigh-Ritz eigensolver did not converge");
    for (int64_t a = 0; a < nact; ++a) lam_act[a] = static_cast<double>(lam_dev[a]);
    for (int64_t a = 0; a < nact; ++a)
      if (!std::isfinite(lam_act[a]) || !std::isfinite(res_act[a]))
        return set_error(ctx_, CHASE_ENUMERIC, "NaN/Inf in Ritz values or residuals");

    // DEFLATION & LOCKING (Alg. 3): Ritz values arrive ascending from zheevd.
    std::vector<int> order(nact);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return lam_act[x] < lam_act[y]; });
    int64_t n_new = 0;
    while (n_new < nact && res_act[order[n_new]] <= tol_eff) ++n_new;
    for (int64_t q = 0; q < n_new; ++q) {
      lam_lock.push_back(lam_act[order[q]]);
      res_lock.push_back(res_act[order[q]]);
    }
    // interval update
    double lo = INFINITY, hi = -INFINITY;
    for (double x : lam_lock) lo = std::min(lo, x), hi = std::max(hi, x);
    for (int64_t a = 0; a < nact; ++a) lo = std::min(lo, lam_act[a]), hi = std::max(hi, lam_act[a]);
    mu_1_ = lo;
    mu_b_ = hi;
    if (!(mu_b_ < b_sup_)) mu_b_ = b_sup_ - 1e-12 * std::fabs(b_sup_) - 1e-300;
    const double c = 0.5 * (b_sup_ + mu_b_), e = 0.5 * (b_sup_ - mu_b_);
    // degrees (Alg. 5) and precision groups
    const int64_t rem = nact - n_new;
    std::vector<int> mnew(rem), pnew(rem), idx(rem);
    std::vector<double> nres(rem);
    std::vector<char> nfp32(rem), nl64(rem);
    for (int64_t q = 0; q < rem; ++q) {
      const int64_t r = n_new + q;
      const int a = order[r];
      const bool stuck = mixed && hist_fp32[r] && res_act[a] > 0.5 * hist_res[r];
      const bool l64 = lock64[r] || stuck;
      const bool fp32 = mixed && !l64 && res_act[a] > tol32;
      pnew[q] = fp32 ? 1 : 0;
      nres[q] = res_act[a];
      nfp32[q] = fp32 ? 1 : 0;
      nl64[q] = l64 ? 1 : 0;
      if (cfg_.optim)
        mnew[q] = fp32 ? degree_of(tol32, res_act[a], lam_act[a], c, e, cfg_.deg_extra, deg32max)
                       : degree_of(tol_eff, res_act[a], lam_act[a], c, e, cfg_.deg_extra,
                                   cfg_.deg_max);
      else
        mnew[q] = fp32 ? std::min(deg0, deg32max) : deg0;
      idx[q] = static_cast<int>(q);
    }
    for (int64_t q = 0; q < rem; ++q) {
      hist_res[q] = nres[q];
      hist_fp32[q] = nfp32[q];
      lock64[q] = nl64[q];
    }
    // sort: key (precision group: FP32 first, degree)
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
      if (pnew[x] != pnew[y]) return pnew[x] > pnew[y];
      return mnew[x] < mnew[y];
    });
    std::vector<double> la2(nb_), re2(nb_);
    for (int64_t q = 0; q < n_new; ++q) perm[q] = order[q];
    for (int64_t q = 0; q < rem; ++q) {
      perm[n_new + q] = order[n_new + idx[q]];
      m[q] = mnew[idx[q]];
      prec[q] = pnew[idx[q]];
      la2[q] = lam_act[order[n_new + idx[q]]];
      re2[q] = res_act[order[n_new + idx[q]]];
    }
    for (int64_t q = 0; q < rem; ++q) lam_act[q] = la2[q], res_act[q] = re2[q];
    // apply the order on the device: W <- V[:, perm], V <- W
    if ((rc = hip(hipMemcpyAsync(at<int>(L_.perm), perm.data(), nact * 4, hipMemcpyHostToDevice, s_),
                  "h2d")))
      return rc;
    if ((rc = hip(launch_gather(Q, n_, Wb, n_, n_, at<int>(L_.perm), nact, s_, w_), "gather")))
      return rc;
    if ((rc = hip(hipMemcpyAsync(Q, Wb, static_cast<size_t>(n_) * nact * es(),
                                 hipMemcpyDeviceToDevice, s_),
                  "copy")))
      return rc;
    nlock += n_new;
    if (cfg_.verbose) {
      int64_t n32 = 0;
      double rmax = 0.0;
      for (int64_t q = 0; q < rem; ++q) n32 += prec[q], rmax = std::max(rmax, res_act[q]);
      const double secs =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
      std::fprintf(stderr,
                   "chase: iteration %d: locked %lld of %lld, largest active residual %.3e "
                   "(tol %.3e), next filter: %lld FP32 columns, degrees %d..%d, %.2f s\n",
                   it, static_cast<long long>(nlock), static_cast<long long>(cfg_.nev), rmax,
                   tol_eff, static_cast<long long>(n32), rem > 0 ? m[0] : 0,
                   rem > 0 ? *std::max_element(m.begin(), m.begin() + rem) : 0, secs);
      std::fflush(stderr);
    }
  }

  // ---------------------------------------------------------------- output
  const int64_t nact = nb_ - nlock;
  std::vector<int> lo_idx(nlock), ac_idx(nact);
  std::iota(lo_idx.begin(), lo_idx.end(), 0);
  std::iota(ac_idx.begin(), ac_idx.end(), 0);
  std::stable_sort(lo_idx.begin(), lo_idx.end(), [&](int x, int y) { return lam_lock[x] < lam_lock[y]; });
  std::stable_sort(ac_idx.begin(), ac_idx.end(), [&](int x, int y) { return lam_act[x] < lam_act[y]; });
  for (int64_t q = 0; q < nlock; ++q) {
    perm[q] = lo_idx[q];
    ritzv[q] = lam_lock[lo_idx[q]];
    resid[q] = res_lock[lo_idx[q]];
  }
  for (int64_t q = 0; q < nact; ++q) {
    perm[nlock + q] = static_cast<int>(nlock) + ac_idx[q];
    ritzv[nlock + q] = lam_act[ac_idx[q]];
    resid[nlock + q] = res_act[ac_idx[q]];
  }
  if ((rc = hip(hipMemcpyAsync(at<int>(L_.perm), perm.data(), nb_ * 4, hipMemcpyHostToDevice, s_),
                "h2d")))
    return rc;
  if ((rc = hip(launch_gather(at<R>(L_.V), n_, at<R>(L_.W), n_, n_, at<int>(L_.perm), nb_,
                              s_, w_),
                "gather")))
    return rc;
  if ((rc = hip(hipMemcpy2DAsync(Vuser, ldv * es(), at<R>(L_.W), n_ * es(), n_ * es(), nb_,
                                 hipMemcpyDeviceToDevice, s_),
                "copy out")))
    return rc;
  (void)hipEventRecord(ev[7], s_);
  if ((rc = hip(hipStreamSynchronize(s_), "sync"))) return rc;
  st_.total_ms = elapsed(6, 7);
  st_.iterations = it;
  st_.nconv = static_cast<int32_t>(nlock);
  st_.qr_fallbacks = fallbacks_;
  st_.matvecs += st_.filter_matvecs;
  // 8 n^2 flops per complex matvec, 2 n^2 per real one
  st_.filter_flops = (real_ ? 2.0 : 8.0) * static_cast<double>(n_) * static_cast<double>(n_) *
                     static_cast<double>(st_.filter_matvecs);
  st_.b_sup = b_sup_;
  st_.mu_1 = mu_1_;
  st_.mu_nevnex = mu_b_;
  st_.norm_est = norm_est_;
  st_.status = nlock >= cfg_.nev ? CHASE_OK : CHASE_NOT_CONVERGED;
  if (stats) *stats = st_;
  return st_.status;
}

}  // namespace

int check_config(chase_ctx* ctx, const chase_config* cfg) {
  if (!cfg) return set_error(ctx, CHASE_EINVAL, "cfg is NULL");
  if (cfg->n < 1 || cfg->nev < 1 || cfg->nex < 0 || cfg->nev + cfg->nex > cfg->n)
    return set_error(ctx, CHASE_EINVAL, "need n >= 1, nev >= 1, nex >= 0, nev + nex <= n");
  if (cfg->n > 0x7fffffffLL) return set_error(ctx, CHASE_EINVAL, "n must fit in int32");
  if (!(cfg->tol > 0.0) || !std::isfinite(cfg->tol))
    return set_error(ctx, CHASE_EINVAL, "tol must be positive");
  if (cfg->deg < 1 || cfg->deg > 64 || cfg->deg_max < 2 || cfg->deg_max > 64 || cfg->deg_extra < 0)
    return set_error(ctx, CHASE_EINVAL, "deg in [1, 64], deg_max in [2, 64], deg_extra >= 0");
  if (cfg->max_iter < 1) return set_error(ctx, CHASE_EINVAL, "max_iter must be >= 1");
  if (cfg->lanczos_iter < 1 || cfg->num_lanczos < 1)
    return set_error(ctx, CHASE_EINVAL, "lanczos_iter and num_lanczos must be >= 1");
  if (cfg->precision != CHASE_FP64 && cfg->precision != CHASE_MIXED &&
      cfg->precision != CHASE_FP32)
    return set_error(ctx, CHASE_EINVAL, "precision must be CHASE_FP64, CHASE_FP32 or CHASE_MIXED");
  if (cfg->precision == CHASE_MIXED &&
      (!(cfg->switch_resid > 0.0) || cfg->deg_max_fp32 < 2 || cfg->deg_max_fp32 > 64))
    return set_error(ctx, CHASE_EINVAL, "switch_resid > 0 and deg_max_fp32 in [2, 64]");
  if (!(cfg->dos_sigma > 0.0)) return set_error(ctx, CHASE_EINVAL, "dos_sigma must be positive");
  if (cfg->real_symmetric != 0 && cfg->real_symmetric != 1)
    return set_error(ctx, CHASE_EINVAL, "real_symmetric must be 0 or 1");
  if (cfg->filter_3m != 0 && cfg->filter_3m != 1)
    return set_error(ctx, CHASE_EINVAL, "filter_3m must be 0 or 1");
  if (cfg->have_mu && !cfg->approx &&
      !(std::isfinite(cfg->mu_1) && std::isfinite(cfg->mu_nevnex) && cfg->mu_1 < cfg->mu_nevnex))
    return set_error(ctx, CHASE_EINVAL, "need finite mu_1 < mu_nevnex");
  return CHASE_OK;
}

int solve_with(chase_ctx* ctx, const chase_config* cfg, const void* H, int64_t ldh, void* V,
               int64_t ldv, double* ritzv, double* resid, chase_stats* stats, Batcher* batcher) {
  if (!ctx) return CHASE_EINVAL;
  ctx->last_error.clear();
  int rc = check_config(ctx, cfg);
  if (rc) return rc;
  if (!H || !V || !ritzv || !resid) return set_error(ctx, CHASE_EINVAL, "NULL buffer");
  if (ldh < cfg->n || ldv < cfg->n) return set_error(ctx, CHASE_EINVAL, "leading dimension < n");
  const int64_t nb = cfg->nev + cfg->nex;
  if (cfg->approx)
    for (int64_t i = 0; i < nb; ++i)
      if (!std::isfinite(ritzv[i])) return set_error(ctx, CHASE_EINVAL, "ritzv must be finite");
  const char* ph = static_cast<const char*>(H);
  const char* pv = static_cast<const char*>(V);
  const size_t es = solve_elem_bytes(*cfg);
  const size_t hb = (static_cast<size_t>(cfg->n - 1) * ldh + cfg->n) * es;
  const size_t vb = (static_cast<size_t>(nb - 1) * ldv + cfg->n) * es;
  if (ph < pv + vb && pv < ph + hb) return set_error(ctx, CHASE_EINVAL, "H and V overlap");
  if ((rc = hip_ok(ctx))) return rc;
  if (cfg->precision == CHASE_FP32) {  // products never batched: the batcher groups FP64 work
    Solver<float> s(ctx, *cfg, nullptr);
    return s.run(H, ldh, V, ldv, ritzv, resid, stats);
  }
  Solver<double> s(ctx, *cfg, batcher);
  return s.run(H, ldh, V, ldv, ritzv, resid, stats);
}

hipError_t launch_start_block(void* V, const chase_config& c, uint64_t seed, hipStream_t s) {
  const int64_t nb = c.nev + c.nex;
  if (c.precision == CHASE_FP32)
    return launch_gaussian(static_cast<float*>(V), c.n, c.n, nb, seed, s, solve_width(c));
  return launch_gaussian(static_cast<double*>(V), c.n, c.n, nb, seed, s, solve_width(c));
}

int hip_ok(chase_ctx* ctx) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess)
    return set_error(ctx, CHASE_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
  return CHASE_OK;
}

}  // namespace chase

struct chase_seq {
  chase_ctx* ctx = nullptr;
  chase_config cfg{};
  void* V = nullptr;  // n x (nev + nex), ld n, device resident between problems
  std::vector<double> ritzv;
  int64_t solved = 0;
};

using namespace chase;

extern "C" {

size_t chase_workspace_bytes(const chase_config* cfg) {
  if (!cfg || cfg->n <= 0 || cfg->nev <= 0) return 0;
  const int64_t nb = cfg->nev + cfg->nex;
  const int64_t nv = cfg->approx ? 1 : 1 + std::max<int64_t>(cfg->num_lanczos, 1);
  const int64_t k = std::min<int64_t>(std::max(cfg->lanczos_iter, 1), cfg->n);
  const bool planar64 =
      cfg->precision != CHASE_FP32 && !cfg->real_symmetric && cfg->filter_3m != 0;
  return make_layout(cfg->n, nb, nv, k, cfg->precision == CHASE_MIXED, solve_width(*cfg),
                     solve_scalar_bytes(*cfg), planar64).total;
}

int chase_solve(chase_ctx* ctx, const chase_config* cfg, const void* H, int64_t ldh, void* V,
                int64_t ldv, double* ritzv, double* resid, chase_stats* stats) {
  return solve_with(ctx, cfg, H, ldh, V, ldv, ritzv, resid, stats, nullptr);
}

int chase_seq_create(chase_ctx* ctx, const chase_config* cfg, chase_seq** out) {
  if (!ctx || !out) return CHASE_EINVAL;
  *out = nullptr;
  int rc = check_config(ctx, cfg);
  if (rc) return rc;
  if ((rc = hip_ok(ctx))) return rc;
  chase_seq* s = new chase_seq();
  s->ctx = ctx;
  s->cfg = *cfg;
  const int64_t nb = cfg->nev + cfg->nex;
  if (hipMalloc(&s->V, static_cast<size_t>(cfg->n) * nb * solve_elem_bytes(*cfg)) != hipSuccess) {
    (void)hipGetLastError();
    delete s;
    return set_error(ctx, CHASE_ENOMEM, "sequence state allocation failed");
  }
  // start block of problem 1: counter-based Gaussian from the seed
  hipError_t e = launch_start_block(s->V, *cfg, cfg->seed ^ 0x5eedULL, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    (void)hipFree(s->V);
    delete s;
    return set_error(ctx, CHASE_EDEVICE, std::string("sequence init: ") + hipGetErrorString(e));
  }
  s->ritzv.assign(nb, 0.0);
  *out = s;
  return CHASE_OK;
}

int chase_seq_solve(chase_seq* seq, const void* H, int64_t ldh, double* ritzv, double* resid,
                    chase_stats* stats) {
  if (!seq) return CHASE_EINVAL;
  chase_config cfg = seq->cfg;
  cfg.approx = seq->solved > 0 ? 1 : seq->cfg.approx;
  if (cfg.approx) cfg.have_mu = 0;
  std::vector<double> rv = seq->ritzv;
  const int64_t nb = cfg.nev + cfg.nex;
  std::vector<double> rs(nb, 0.0);
  if (seq->solved == 0 && seq->cfg.approx && ritzv) rv.assign(ritzv, ritzv + nb);
  int rc = solve_with(seq->ctx, &cfg, H, ldh, seq->V, cfg.n, rv.data(), rs.data(), stats, nullptr);
  if (rc < 0) return rc;
  seq->ritzv = rv;
  ++seq->solved;
  if (ritzv) std::copy(rv.begin(), rv.end(), ritzv);
  if (resid) std::copy(rs.begin(), rs.end(), resid);
  return rc;
}

int chase_seq_vectors(chase_seq* seq, void** V, int64_t* ldv) {
  if (!seq || !V || !ldv) return CHASE_EINVAL;
  *V = seq->V;
  *ldv = seq->cfg.n;
  return CHASE_OK;
}

void chase_seq_destroy(chase_seq* seq) {
  if (!seq) return;
  (void)hipSetDevice(seq->ctx->device);
  (void)hipStreamSynchronize(seq->ctx->stream);
  if (seq->V) (void)hipFree(seq->V);
  delete seq;
}

}  // extern "C"
