// Small kernels of the outer loop (Algorithm 1): Lanczos vector updates (Alg. 6), column
// normalisation, residual norms (Alg. 1), column gathers for locking and sorting
// (Alg. 1, Alg. 3), Hermitian symmetrisation of the Rayleigh quotient (Alg. 2) and a
// counter-based Gaussian generator for Lanczos start vectors.
//
// Every reduction runs in one workgroup per column with a fixed-order tree, so results are
// bitwise reproducible from run to run (no atomics).

#include "internal.h"

#include <type_traits>

namespace chase {
namespace {

constexpr int RT = 256;  // threads per column block

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = RT / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Kernels are templated on the scalar R of the vectors (double or float) and on W, the values per
// element: 2 for interleaved complex data, 1 for real data.  Reductions accumulate in double.

// Column c of a Lanczos block step:  w <- w - beta_prev u_prev;  alpha = Re(u^H w);
// w <- w - alpha u;  beta = ||w||;  u_next = w / beta.
template <typename R, int W>
__global__ void lanczos_step_kernel(const R* __restrict__ U, const R* __restrict__ Up,
                                    R* __restrict__ Wv, R* __restrict__ Un, int64_t n,
                                    int64_t ld, const double* __restrict__ beta_prev,
                                    double* __restrict__ alpha_out,
                                    double* __restrict__ beta_out) {
  __shared__ double sh[RT];
  const int c = blockIdx.x;
  const R* u = U + W * c * ld;
  const R* up = Up + W * c * ld;
  R* w = Wv + W * c * ld;
  R* un = Un + W * c * ld;
  const double bp = beta_prev[c];
  const int64_t m = W * n;  // values of one column
  double part = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += RT) {
    const R x = static_cast<R>(w[i] - bp * up[i]);
    w[i] = x;
    part += static_cast<double>(u[i]) * x;
  }
  const double alpha = block_sum(part, sh);
  part = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += RT) {
    const R x = static_cast<R>(w[i] - alpha * u[i]);
    w[i] = x;
    part += static_cast<double>(x) * x;
  }
  const double beta = sqrt(block_sum(part, sh));
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int64_t i = threadIdx.x; i < m; i += RT) un[i] = static_cast<R>(w[i] * inv);
  if (threadIdx.x == 0) {
    alpha_out[c] = alpha;
    beta_out[c] = beta;
  }
}

template <typename R, int W>
__global__ void normalize_kernel(R* __restrict__ X, int64_t n, int64_t ld) {
  __shared__ double sh[RT];
  R* x = X + W * blockIdx.x * ld;
  const int64_t m = W * n;
  double part = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += RT) part += static_cast<double>(x[i]) * x[i];
  const double nrm = sqrt(block_sum(part, sh));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t i = threadIdx.x; i < m; i += RT) x[i] = static_cast<R>(x[i] * inv);
}

// r_a = || AV_a - lambda_a V_a ||_2
template <typename R, int W>
__global__ void resid_kernel(const R* __restrict__ AV, const R* __restrict__ V,
                             const R* __restrict__ lam, int64_t n, int64_t ld,
                             double* __restrict__ out) {
  __shared__ double sh[RT];
  const int c = blockIdx.x;
  const R* a = AV + W * c * ld;
  const R* v = V + W * c * ld;
  const double l = lam[c];
  const int64_t m = W * n;
  double part = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += RT) {
    const double d = static_cast<double>(a[i]) - l * v[i];
    part += d * d;
  }
  const double r = sqrt(block_sum(part, sh));
  if (threadIdx.x == 0) out[c] = r;
}

template <typename R, int W>
__global__ void gather_kernel(const R* __restrict__ src, int64_t lds, R* __restrict__ dst,
                              int64_t ldd, int64_t n, const int* __restrict__ perm) {
  using R2 = typename std::conditional<sizeof(R) == 8, double2, float2>::type;
  const int c = blockIdx.y;
  const R* s = src + W * static_cast<int64_t>(perm[c]) * lds;
  R* d = dst + W * static_cast<int64_t>(c) * ldd;
  if constexpr (W == 2) {
    const R2* s2 = reinterpret_cast<const R2*>(s);
    R2* d2 = reinterpret_cast<R2*>(d);
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
      d2[i] = s2[i];
  } else {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
      d[i] = s[i];
  }
}

// G <- (G + G^H) / 2 on an m x m matrix (complex Hermitian part, or real symmetric part)
template <typename R, int W>
__global__ void herm_sym_kernel(R* __restrict__ G, int64_t ld, int64_t m) {
  const int64_t total = m * m;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i = t % m, j = t / m;
    if (i > j) continue;
    R* a = G + W * (i + j * ld);
    R* b = G + W * (j + i * ld);
    if constexpr (W == 2) {
      if (i == j) {
        a[1] = R(0);
      } else {
        const R re = R(0.5) * (a[0] + b[0]);
        const R im = R(0.5) * (a[1] - b[1]);
        a[0] = re;
        a[1] = im;
        b[0] = re;
        b[1] = -im;
      }
    } else if (i != j) {
      const R v = R(0.5) * (a[0] + b[0]);
      a[0] = v;
      b[0] = v;
    }
  }
}

template <typename R, int W>
__global__ void add_diag_kernel(R* __restrict__ G, int64_t ld, int64_t m, double s) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < m) G[W * (i + i * ld)] += static_cast<R>(s);
}

// G = sum over s of the slices P_s (m1 x m2 elements, ld m1, stride elements apart), summed in
// FP64 in slice order; one thread per scalar of G.
template <typename R, int W>
__global__ void sum_slices_kernel(const R* __restrict__ P, int64_t m1, int64_t m2, int64_t stride,
                                  int p, R* __restrict__ G, int64_t ldg) {
  const int64_t rows = W * m1, total = rows * m2;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = t % rows, c = t / rows;
    double acc = 0.0;
    for (int q = 0; q < p; ++q) acc += static_cast<double>(P[W * stride * q + r + c * rows]);
    G[r + c * W * ldg] = static_cast<R>(acc);
  }
}

// Interleaved complex64 n x n (ld lds) -> planar: Re plane at dst, Im plane at dst + ldd * n.
__global__ void split_planes_kernel(const float* __restrict__ src, int64_t lds,
                                    float* __restrict__ dst, int64_t ldd, int64_t n) {
  const int64_t total = n * n;
  float* im = dst + ldd * n;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = t % n, c = t / n;
    const float2 v = *reinterpret_cast<const float2*>(src + 2 * (r + c * lds));
    dst[r + c * ldd] = v.x;
    im[r + c * ldd] = v.y;
  }
}

// SplitMix64 (Steele, Lea, Flood 2014) applied to a counter, then Box-Muller.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

template <typename R, int W>
__global__ void gaussian_kernel(R* __restrict__ X, int64_t n, int64_t ld, int64_t cols,
                                uint64_t seed) {
  const int64_t total = n * cols;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i = t % n, c = t / n;
    const uint64_t k = splitmix64(seed ^ splitmix64(static_cast<uint64_t>(c * n + i)));
    const uint64_t k2 = splitmix64(k);
    const double u1 = (static_cast<double>(k >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = static_cast<double>(k2 >> 11) * (1.0 / 9007199254740992.0);
    const double r = sqrt(-2.0 * log(u1));
    X[W * (i + c * ld)] = static_cast<R>(r * cos(6.283185307179586 * u2));
    if constexpr (W == 2) X[W * (i + c * ld) + 1] = static_cast<R>(r * sin(6.283185307179586 * u2));
  }
}

unsigned grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 32768) b = 32768;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

#define CHASE_BY_W(w, R, K) ((w) == 1 ? K<R, 1> : K<R, 2>)

template <typename R>
hipError_t lanczos_step_t(const R* U, const R* Up, R* W, R* Un, int64_t n, int64_t ld, int64_t nv,
                          const double* beta_prev, double* alpha_out, double* beta_out,
                          hipStream_t s, int w) {
  hipLaunchKernelGGL(CHASE_BY_W(w, R, lanczos_step_kernel), dim3(static_cast<unsigned>(nv)),
                     dim3(RT), 0, s, U, Up, W, Un, n, ld, beta_prev, alpha_out, beta_out);
  return hipGetLastError();
}
template <typename R>
hipError_t normalize_t(R* X, int64_t n, int64_t ld, int64_t cols, hipStream_t s, int w) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(CHASE_BY_W(w, R, normalize_kernel), dim3(static_cast<unsigned>(cols)),
                     dim3(RT), 0, s, X, n, ld);
  return hipGetLastError();
}
template <typename R>
hipError_t resid_t(const R* AV, const R* V, const R* lam, int64_t n, int64_t ld, int64_t cols,
                   double* out, hipStream_t s, int w) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(CHASE_BY_W(w, R, resid_kernel), dim3(static_cast<unsigned>(cols)), dim3(RT),
                     0, s, AV, V, lam, n, ld, out);
  return hipGetLastError();
}
template <typename R>
hipError_t gather_t(const R* src, int64_t lds, R* dst, int64_t ldd, int64_t n, const int* perm,
                    int64_t cols, hipStream_t s, int w) {
  if (cols <= 0) return hipSuccess;
  unsigned gx = static_cast<unsigned>((n + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(CHASE_BY_W(w, R, gather_kernel), dim3(gx, static_cast<unsigned>(cols)),
                     dim3(256), 0, s, src, lds, dst, ldd, n, perm);
  return hipGetLastError();
}
template <typename R>
hipError_t herm_sym_t(R* G, int64_t ld, int64_t m, hipStream_t s, int w) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(CHASE_BY_W(w, R, herm_sym_kernel), dim3(grid_for(m * m)), dim3(256), 0, s, G,
                     ld, m);
  return hipGetLastError();
}
template <typename R>
hipError_t add_diag_t(R* G, int64_t ld, int64_t m, double v, hipStream_t s, int w) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(CHASE_BY_W(w, R, add_diag_kernel), dim3(grid_for(m)), dim3(256), 0, s, G, ld,
                     m, v);
  return hipGetLastError();
}
template <typename R>
hipError_t sum_slices_t(const R* P, int64_t m1, int64_t m2, int64_t stride, int p, R* G,
                        int64_t ldg, hipStream_t s, int w) {
  if (m1 <= 0 || m2 <= 0) return hipSuccess;
  hipLaunchKernelGGL(CHASE_BY_W(w, R, sum_slices_kernel), dim3(grid_for(w * m1 * m2)), dim3(256),
                     0, s, P, m1, m2, stride, p, G, ldg);
  return hipGetLastError();
}
template <typename R>
hipError_t gaussian_t(R* X, int64_t n, int64_t ld, int64_t cols, uint64_t seed, hipStream_t s,
                      int w) {
  if (cols <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(CHASE_BY_W(w, R, gaussian_kernel), dim3(grid_for(n * cols)), dim3(256), 0, s,
                     X, n, ld, cols, seed);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_split_planes_c64(const float* src, int64_t lds, float* dst, int64_t ldd,
                                   int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_planes_kernel, dim3(grid_for(n * n)), dim3(256), 0, s, src, lds, dst,
                     ldd, n);
  return hipGetLastError();
}

#define CHASE_LOOP_API(R)                                                                       \
  hipError_t launch_lanczos_step(const R* U, const R* Up, R* W, R* Un, int64_t n, int64_t ld,   \
                                 int64_t nv, const double* bp, double* ao, double* bo,          \
                                 hipStream_t s, int w) {                                        \
    return lanczos_step_t<R>(U, Up, W, Un, n, ld, nv, bp, ao, bo, s, w);                         \
  }                                                                                             \
  hipError_t launch_normalize(R* X, int64_t n, int64_t ld, int64_t cols, hipStream_t s, int w) { \
    return normalize_t<R>(X, n, ld, cols, s, w);                                                \
  }                                                                                             \
  hipError_t launch_resid(const R* AV, const R* V, const R* lam, int64_t n, int64_t ld,         \
                          int64_t cols, double* out, hipStream_t s, int w) {                    \
    return resid_t<R>(AV, V, lam, n, ld, cols, out, s, w);                                      \
  }                                                                                             \
  hipError_t launch_gather(const R* src, int64_t lds, R* dst, int64_t ldd, int64_t n,           \
                           const int* perm, int64_t cols, hipStream_t s, int w) {               \
    return gather_t<R>(src, lds, dst, ldd, n, perm, cols, s, w);                                \
  }                                                                                             \
  hipError_t launch_herm_sym(R* G, int64_t ld, int64_t m, hipStream_t s, int w) {               \
    return herm_sym_t<R>(G, ld, m, s, w);                                                       \
  }                                                                                             \
  hipError_t launch_add_diag(R* G, int64_t ld, int64_t m, double v, hipStream_t s, int w) {     \
    return add_diag_t<R>(G, ld, m, v, s, w);                                                    \
  }                                                                                             \
  hipError_t launch_sum_slices(const R* P, int64_t m1, int64_t m2, int64_t stride, int p, R* G,  \
                              int64_t ldg, hipStream_t s, int w) {                              \
    return sum_slices_t<R>(P, m1, m2, stride, p, G, ldg, s, w);                                 \
  }                                                                                             \
  hipError_t launch_gaussian(R* X, int64_t n, int64_t ld, int64_t cols, uint64_t seed,          \
                             hipStream_t s, int w) {                                            \
    return gaussian_t<R>(X, n, ld, cols, seed, s, w);                                           \
  }

CHASE_LOOP_API(double)
CHASE_LOOP_API(float)

#undef CHASE_LOOP_API
#undef CHASE_BY_W

}  // namespace chase
