// Cholesky factorisation G = R^H R (R upper triangular, written over the upper triangle of G)
// for the Gram matrices of the CholeskyQR passes of ORTHOGONALIZE.
//
// The vendor factorisation gave results that differed in the last bits from run to run when
// other work shared the device (the same input matrix, a different R), which made a solve's
// outcome depend on what ran beside it.  This blocked right-looking factorisation fixes every
// summation order.  Per block column of width kB it factors the diagonal block in LDS (column
// by column, one barrier per column: the pivot row stays unscaled during the trailing update,
// a_ic -= conj(a_ji) a_jc / a_jj, and the block's rows are scaled at the end), solves the block
// row to its right column by column (one thread per column, forward substitution in a fixed
// order), and subtracts the block row's Gram product from the trailing upper triangle
// (fixed-order sums over the kB rows).  Up to kSmallMax columns one workgroup does all of it in
// a single launch (the block row kept in LDS for the update); beyond, three launches per block.
// Only the upper triangle of G is read or written.
//
// info (device int): 0 on success, else 1 + the index of the first pivot that is not positive
// (or not finite); later block columns then run on garbage that the caller discards.

#include "internal.h"

namespace chase {
namespace {

constexpr int kB = 32;            // block width
constexpr int kCholThreads = 256;  // workgroup of the multi-launch kernels
constexpr int kSmallMax = 256;     // largest order factored by the single-workgroup kernel
constexpr int kSmallThreads = 1024;

// element helpers: complex (W = 2, pairs of T) or real (W = 1)
template <typename T, int W> struct El;
template <typename T> struct El<T, 2> {
  struct V { T re, im; };
  static __device__ __forceinline__ V ld(const T* p) { return V{p[0], p[1]}; }
  static __device__ __forceinline__ void st(T* p, V v) { p[0] = v.re, p[1] = v.im; }
  static __device__ __forceinline__ V zero() { return V{T(0), T(0)}; }
  static __device__ __forceinline__ T real(V v) { return v.re; }
  static __device__ __forceinline__ V from_real(T r) { return V{r, T(0)}; }
  static __device__ __forceinline__ V scale(V v, T s) { return V{v.re * s, v.im * s}; }
  // acc - conj(a) * b
  static __device__ __forceinline__ V sub_conj_mul(V acc, V a, V b) {
    acc.re -= a.re * b.re + a.im * b.im;
    acc.im -= a.re * b.im - a.im * b.re;
    return acc;
  }
};
template <typename T> struct El<T, 1> {
  using V = T;
  static __device__ __forceinline__ V ld(const T* p) { return *p; }
  static __device__ __forceinline__ void st(T* p, V v) { *p = v; }
  static __device__ __forceinline__ V zero() { return T(0); }
  static __device__ __forceinline__ T real(V v) { return v; }
  static __device__ __forceinline__ V from_real(T r) { return r; }
  static __device__ __forceinline__ V scale(V v, T s) { return v * s; }
  static __device__ __forceinline__ V sub_conj_mul(V acc, V a, V b) { return acc - a * b; }
};

// Factor the b x b block held in A (upper triangle; rows and columns relative to the block) in
// place: A <- R.  NT threads; the caller has synchronised after loading A.  piv receives the
// pivots' square roots (0 for a pivot that is not positive or not finite); *bad (LDS, set to 0
// by the caller) receives 1 + the first such pivot's index.
template <typename T, int W, int NT>
__device__ __forceinline__ void factor_block(typename El<T, W>::V (&A)[kB][kB + 1], T (&piv)[kB],
                                             int b, int* bad) {
  using E = El<T, W>;
  const int tid = threadIdx.x;
  for (int j = 0; j < b; ++j) {
    // the imaginary part of a Hermitian diagonal is dropped
    const T d = E::real(A[j][j]);
    const bool ok = d > T(0) && isfinite(d);
    if (tid == 0) {
      if (!ok && !*bad) *bad = j + 1;
      piv[j] = ok ? sqrt(d) : T(0);
    }
    const T dinv = ok ? T(1) / d : T(0);
    // trailing upper triangle with the unscaled row j: A[i][c] -= conj(A[j][i]) A[j][c] / d
    const int rem = b - j - 1;
    for (int e = tid; e < rem * rem; e += NT) {
      const int i = j + 1 + e % rem, c = j + 1 + e / rem;
      if (i <= c) A[i][c] = E::sub_conj_mul(A[i][c], E::scale(A[j][i], dinv), A[j][c]);
    }
    __syncthreads();
  }
  // rows scaled by their pivots: R[i][c] = A[i][c] / sqrt(d_i), R[i][i] = sqrt(d_i)
  for (int e = tid; e < b * b; e += NT) {
    const int i = e % b, c = e / b;
    if (i < c) A[i][c] = E::scale(A[i][c], piv[i] > T(0) ? T(1) / piv[i] : T(0));
    else if (i == c) A[i][i] = E::from_real(piv[i]);
  }
  __syncthreads();
}

// Column c (absolute) of the block row right of the diagonal block at k:
// y = R_kk^{-H} G[k:k+b, c] by forward substitution with the lower triangular R_kk^H, written
// back to G; returned in y.
template <typename T, int W>
__device__ __forceinline__ void panel_column(T* __restrict__ G, int64_t ldg, int k, int b, int c,
                                             const typename El<T, W>::V (&R)[kB][kB + 1],
                                             typename El<T, W>::V (&y)[kB]) {
  using E = El<T, W>;
  using V = typename E::V;
  T* col = G + W * (static_cast<int64_t>(c) * ldg);
#pragma unroll
  for (int i = 0; i < kB; ++i) {
    if (i < b) {
      V acc = E::ld(col + W * (k + i));
#pragma unroll
      for (int j = 0; j < kB; ++j)
        if (j < i) acc = E::sub_conj_mul(acc, R[j][i], y[j]);
      const T d = E::real(R[i][i]);
      y[i] = E::scale(acc, d > T(0) ? T(1) / d : T(0));
    }
  }
#pragma unroll
  for (int i = 0; i < kB; ++i)
    if (i < b) E::st(col + W * (k + i), y[i]);
}

// The b x b diagonal block at (k, k), for the multi-launch path.
template <typename T, int W>
__global__ __launch_bounds__(kCholThreads) void chol_diag_kernel(T* __restrict__ G, int64_t ldg,
                                                                 int k, int b, int* info) {
  using E = El<T, W>;
  using V = typename E::V;
  __shared__ V A[kB][kB + 1];  // A[i][c]: row i, column c of the block (upper part used)
  __shared__ T piv[kB];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) {
    bad = 0;
    if (k == 0) *info = 0;
  }
  for (int e = tid; e < b * b; e += kCholThreads) {
    const int i = e % b, c = e / b;
    A[i][c] = i <= c ? E::ld(G + W * ((k + i) + static_cast<int64_t>(k + c) * ldg)) : E::zero();
  }
  __syncthreads();
  factor_block<T, W, kCholThreads>(A, piv, b, &bad);
  for (int e = tid; e < b * b; e += kCholThreads) {
    const int i = e % b, c = e / b;
    if (i <= c) E::st(G + W * ((k + i) + static_cast<int64_t>(k + c) * ldg), A[i][c]);
  }
  if (tid == 0 && bad && *info == 0) *info = k + bad;
}

// The whole factorisation of an m x m matrix, m <= kSmallMax, in one workgroup.
template <typename T, int W>
__global__ __launch_bounds__(kSmallThreads) void chol_small_kernel(T* __restrict__ G, int64_t ldg,
                                                                   int m, int* info) {
  using E = El<T, W>;
  using V = typename E::V;
  constexpr int NT = kSmallThreads;
  __shared__ V A[kB][kB + 1];
  __shared__ V P[kB][kSmallMax - kB];  // block row right of the diagonal block
  __shared__ T piv[kB];
  __shared__ int bad, first;
  const int tid = threadIdx.x;
  if (tid == 0) first = 0;
  for (int k = 0; k < m; k += kB) {
    const int b = m - k < kB ? m - k : kB;
    if (tid == 0) bad = 0;
    for (int e = tid; e < b * b; e += NT) {
      const int i = e % b, c = e / b;
      A[i][c] = i <= c ? E::ld(G + W * ((k + i) + static_cast<int64_t>(k + c) * ldg)) : E::zero();
    }
    __syncthreads();
    factor_block<T, W, NT>(A, piv, b, &bad);
    for (int e = tid; e < b * b; e += NT) {
      const int i = e % b, c = e / b;
      if (i <= c) E::st(G + W * ((k + i) + static_cast<int64_t>(k + c) * ldg), A[i][c]);
    }
    if (tid == 0 && bad && !first) first = k + bad;
    const int r = m - k - b;
    if (r <= 0) break;
    // block row by forward substitution, one thread per column, the solution kept in P (each
    // thread reads back only its own column)
    for (int c = tid; c < r; c += NT) {
      T* col = G + W * (static_cast<int64_t>(k + b + c) * ldg);
      for (int i = 0; i < b; ++i) {
        V acc = E::ld(col + W * (k + i));
        for (int j = 0; j < i; ++j) acc = E::sub_conj_mul(acc, A[j][i], P[j][c]);
        const T d = E::real(A[i][i]);
        P[i][c] = E::scale(acc, d > T(0) ? T(1) / d : T(0));
      }
      for (int i = 0; i < b; ++i) E::st(col + W * (k + i), P[i][c]);
    }
    __syncthreads();
    // trailing upper triangle: G[i][c] -= sum_l conj(P[l][i]) P[l][c], i <= c, in l order
    for (int e = tid; e < r * r; e += NT) {
      const int i = e % r, c = e / r;
      if (i > c) continue;
      T* g = G + W * ((k + b + i) + static_cast<int64_t>(k + b + c) * ldg);
      V acc = E::ld(g);
      for (int l = 0; l < b; ++l) acc = E::sub_conj_mul(acc, P[l][i], P[l][c]);
      E::st(g, acc);
    }
    __syncthreads();
  }
  if (tid == 0) *info = first;
}

// Block row to the right of the diagonal block: R[k:k+b, c] = R_kk^{-H} G[k:k+b, c] for
// c >= k + b, one thread per column (multi-launch path).
template <typename T, int W>
__global__ __launch_bounds__(kCholThreads) void chol_panel_kernel(T* __restrict__ G, int64_t ldg,
                                                                  int k, int b, int m) {
  using E = El<T, W>;
  using V = typename E::V;
  __shared__ V R[kB][kB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < b * b; e += kCholThreads) {
    const int i = e % b, c = e / b;
    R[i][c] = i <= c ? E::ld(G + W * ((k + i) + static_cast<int64_t>(k + c) * ldg)) : E::zero();
  }
  __syncthreads();
  const int c = k + b + static_cast<int>(blockIdx.x) * kCholThreads + tid;
  if (c >= m) return;
  V y[kB];
  panel_column<T, W>(G, ldg, k, b, c, R, y);
}

// Trailing update of the upper triangle: G[i][c] -= sum_{l < b} conj(R[k+l][i]) R[k+l][c] for
// k + b <= i <= c < m, in 64 x 64 tiles (tiles wholly below the diagonal skipped); each thread
// owns 4 x 4 entries and adds the b terms in order.
template <typename T, int W>
__global__ __launch_bounds__(kCholThreads) void chol_update_kernel(T* __restrict__ G, int64_t ldg,
                                                                   int k, int b, int m) {
  using E = El<T, W>;
  using V = typename E::V;
  constexpr int TT = 64;
  const int base = k + b;
  const int ti = static_cast<int>(blockIdx.x), tc = static_cast<int>(blockIdx.y);
  if (ti > tc) return;
  const int i0 = base + ti * TT, c0 = base + tc * TT;
  __shared__ V Pi[kB][TT + 1];
  __shared__ V Pc[kB][TT + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < b * TT; e += kCholThreads) {
    const int l = e / TT, x = e % TT;
    Pi[l][x] = i0 + x < m ? E::ld(G + W * ((k + l) + static_cast<int64_t>(i0 + x) * ldg)) : E::zero();
    Pc[l][x] = c0 + x < m ? E::ld(G + W * ((k + l) + static_cast<int64_t>(c0 + x) * ldg)) : E::zero();
  }
  __syncthreads();
  const int ri = (tid % 16) * 4, rc = (tid / 16) * 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int i = i0 + ri + a, c = c0 + rc + d;
      if (i >= m || c >= m || i > c) continue;
      T* g = G + W * (i + static_cast<int64_t>(c) * ldg);
      V acc = E::ld(g);
      for (int l = 0; l < b; ++l) acc = E::sub_conj_mul(acc, Pi[l][ri + a], Pc[l][rc + d]);
      E::st(g, acc);
    }
}

template <typename T, int W>
hipError_t potrf_upper(T* G, int64_t ldg, int64_t m, int* info, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (m <= kSmallMax) {
    hipLaunchKernelGGL((chol_small_kernel<T, W>), dim3(1), dim3(kSmallThreads), 0, s, G, ldg,
                       static_cast<int>(m), info);
    return hipGetLastError();
  }
  for (int64_t k = 0; k < m; k += kB) {
    const int b = static_cast<int>(std::min<int64_t>(kB, m - k));
    hipLaunchKernelGGL((chol_diag_kernel<T, W>), dim3(1), dim3(kCholThreads), 0, s, G, ldg,
                       static_cast<int>(k), b, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t r = m - k - b;
    if (r <= 0) continue;
    hipLaunchKernelGGL((chol_panel_kernel<T, W>),
                       dim3(static_cast<unsigned>((r + kCholThreads - 1) / kCholThreads)),
                       dim3(kCholThreads), 0, s, G, ldg, static_cast<int>(k), b,
                       static_cast<int>(m));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned t = static_cast<unsigned>((r + 63) / 64);
    hipLaunchKernelGGL((chol_update_kernel<T, W>), dim3(t, t), dim3(kCholThreads), 0, s, G, ldg,
                       static_cast<int>(k), b, static_cast<int>(m));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_potrf_upper(double* G, int64_t ldg, int64_t m, int* info, hipStream_t s, int w) {
  return w == 2 ? potrf_upper<double, 2>(G, ldg, m, info, s)
                : potrf_upper<double, 1>(G, ldg, m, info, s);
}
hipError_t launch_potrf_upper(float* G, int64_t ldg, int64_t m, int* info, hipStream_t s, int w) {
  return w == 2 ? potrf_upper<float, 2>(G, ldg, m, info, s)
                : potrf_upper<float, 1>(G, ldg, m, info, s);
}

}  // namespace chase
