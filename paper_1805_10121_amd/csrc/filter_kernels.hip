// Chebyshev-filter product kernels for gfx950 (CDNA4).
//
// One launch computes, for the active columns of the block (Alg. 4 lines 4 and 9, Eq. (7)),
//     OUT <- alpha * H X + gamma * X + beta * OUT
// with H complex Hermitian n x n, X and OUT complex n x ncols, all column-major.  The shift
// (A - cI) of Eq. (7) is the gamma = -alpha*c term, so H is never modified.
//
// Complex -> real MFMA mapping (4M real embedding).  The interleaved column-major complex H is,
// byte for byte, a real column-major 2n x n matrix R with R[2i, k] = Re H[i, k] and
// R[2i+1, k] = Im H[i, k].  The B operand is X split into planes [Re X | Im X].  One real
// product R [Re X | Im X] gives, for complex row i and column j,
//     (R ReX)[2i] = ReH ReX,  (R ReX)[2i+1] = ImH ReX,  (R ImX)[2i] = ReH ImX,  (R ImX)[2i+1] = ImH ImX
// and the epilogue combines Re(HX) = ReH ReX - ImH ImX, Im(HX) = ReH ImX + ImH ReX.
// Exactly 8 n^2 ncols real flops; H is read in place, never reformatted.
//
// Tiling: 256 threads (4 waves of 64) own a 64 x 64 complex output tile (128 x 128 real); each
// wave owns 32 x 32 complex = 4 x 4 MFMA 16x16 tiles.  K advances 16 at a time through a
// double-buffered LDS stage fed by a register prefetch of the next stage.
//
// MFMA lane layouts used (16x16x4, checked on gfx950): A operand lane l holds A[l%16][l/16],
// B operand lane l holds B[l/16][l%16].  The accumulator's register r of lane l holds column
// l%16 and row (l/16) + 4r for f64, row 4(l/16) + r for f32.  The A-row permutation below makes
// registers (2p, 2p+1) of a lane the (Re, Im) rows of one complex row for both types, so the
// complex epilogue is lane local.

#include "internal.h"

#include <type_traits>

namespace chase {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> { using type = d4_t; using v2 = double2; };
template <> struct Acc<float> { using type = f4_t; using v2 = float2; };

__device__ __forceinline__ d4_t mfma(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Real row of a 16-row slab that feeds MFMA row i.
template <typename T> __device__ __forceinline__ int a_row(int i);
template <> __device__ __forceinline__ int a_row<double>(int i) {
  // MFMA row i = g + 4r  ->  complex row g + 4*(r/2), part r%2
  return 2 * ((i & 3) + 4 * (i >> 3)) + ((i >> 2) & 1);
}
template <> __device__ __forceinline__ int a_row<float>(int i) { return i; }

// Complex row (0..7 of the slab) held by lane group g in register pair p.
template <typename T> __device__ __forceinline__ int c_row(int g, int p);
template <> __device__ __forceinline__ int c_row<double>(int g, int p) { return g + 4 * p; }
template <> __device__ __forceinline__ int c_row<float>(int g, int p) { return 2 * g + p; }

constexpr int kThreads = 256;
constexpr int BMC = 64;   // complex rows per workgroup tile
constexpr int BNC = 64;   // complex columns per workgroup tile
constexpr int KT = 16;    // K per LDS stage

template <typename T>
__global__ __launch_bounds__(kThreads, 2) void hemm_step_kernel(
    const T* __restrict__ H, int64_t ldh, int n, const T* __restrict__ X, int64_t ldx,
    T* __restrict__ OUT, int64_t ldo, int ncols, T alpha, T beta, T gamma, int tiles_m) {
  using acc_t = typename Acc<T>::type;
  using v2 = typename Acc<T>::v2;
  constexpr int AR = 2 * BMC + 2;  // padded real rows per A stage row (k fixed)
  constexpr int BR = 2 * BNC + 2;  // padded real columns per B stage row (k fixed)
  __shared__ T As[2][KT][AR];
  __shared__ T Bs[2][KT][BR];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int wr = wave >> 1, wc = wave & 1;
  const int tile_m = blockIdx.x % tiles_m, tile_n = blockIdx.x / tiles_m;
  const int i0 = tile_m * BMC, j0 = tile_n * BNC;

  constexpr int A_PER = BMC * KT / kThreads;
  constexpr int B_PER = BNC * KT / kThreads;
  v2 ra[A_PER], rb[B_PER];

  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int q = 0; q < A_PER; ++q) {
      const int idx = tid + kThreads * q;
      const int kk = idx / BMC, ci = idx % BMC;
      const int row = i0 + ci, col = k0 + kk;
      if (row < n && col < n)
        ra[q] = *reinterpret_cast<const v2*>(H + 2 * (static_cast<int64_t>(row) +
                                                       static_cast<int64_t>(col) * ldh));
      else
        ra[q] = v2{T(0), T(0)};
    }
#pragma unroll
    for (int q = 0; q < B_PER; ++q) {
      const int idx = tid + kThreads * q;
      const int jj = idx / KT, kk = idx % KT;
      const int row = k0 + kk, col = j0 + jj;
      if (row < n && col < ncols)
        rb[q] = *reinterpret_cast<const v2*>(X + 2 * (static_cast<int64_t>(row) +
                                                       static_cast<int64_t>(col) * ldx));
      else
        rb[q] = v2{T(0), T(0)};
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int q = 0; q < A_PER; ++q) {
      const int idx = tid + kThreads * q;
      const int kk = idx / BMC, ci = idx % BMC;
      *reinterpret_cast<v2*>(&As[buf][kk][2 * ci]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < B_PER; ++q) {
      const int idx = tid + kThreads * q;
      const int jj = idx / KT, kk = idx % KT;
      Bs[buf][kk][jj] = rb[q].x;
      Bs[buf][kk][BNC + jj] = rb[q].y;
    }
  };

  acc_t acc[4][2][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[a][b][c] = acc_t{0};

  const int arow = a_row<T>(li);
  const int nk = (n + KT - 1) / KT;
  load_tiles(0);
  store_tiles(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load_tiles((kt + 1) * KT);
#pragma unroll
    for (int s = 0; s < KT / 4; ++s) {
      const int k = 4 * s + g;
      T a[4], b[2][2];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) a[rt] = As[cur][k][wr * 64 + rt * 16 + arow];
#pragma unroll
      for (int cg = 0; cg < 2; ++cg) {
        b[cg][0] = Bs[cur][k][wc * 32 + cg * 16 + li];
        b[cg][1] = Bs[cur][k][BNC + wc * 32 + cg * 16 + li];
      }
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int cg = 0; cg < 2; ++cg)
#pragma unroll
          for (int p = 0; p < 2; ++p) acc[rt][cg][p] = mfma(a[rt], b[cg][p], acc[rt][cg][p]);
    }
    if (kt + 1 < nk) store_tiles(cur ^ 1);
    __syncthreads();
  }

  // Epilogue: complex combine, then alpha*HX + gamma*X + beta*OUT.
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int cg = 0; cg < 2; ++cg)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int row = i0 + wr * 32 + rt * 8 + c_row<T>(g, p);
        const int col = j0 + wc * 32 + cg * 16 + li;
        if (row < n && col < ncols) {
          const T hre = acc[rt][cg][0][2 * p] - acc[rt][cg][1][2 * p + 1];
          const T him = acc[rt][cg][1][2 * p] + acc[rt][cg][0][2 * p + 1];
          const v2 x = *reinterpret_cast<const v2*>(
              X + 2 * (static_cast<int64_t>(row) + static_cast<int64_t>(col) * ldx));
          T* o = OUT + 2 * (static_cast<int64_t>(row) + static_cast<int64_t>(col) * ldo);
          T ore = alpha * hre + gamma * x.x;
          T oim = alpha * him + gamma * x.y;
          if (beta != T(0)) {
            const v2 y = *reinterpret_cast<const v2*>(o);
            ore += beta * y.x;
            oim += beta * y.y;
          }
          *reinterpret_cast<v2*>(o) = v2{ore, oim};
        }
      }
}

template <typename S, typename D>
__global__ void convert_kernel(const S* __restrict__ src, int64_t lds, D* __restrict__ dst,
                               int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = t % rows, c = t / rows;
    const S* s = src + 2 * (r + c * lds);
    D* d = dst + 2 * (r + c * ldd);
    d[0] = static_cast<D>(s[0]);
    d[1] = static_cast<D>(s[1]);
  }
}

}  // namespace

template <typename T>
hipError_t launch_hemm_step(const T* H, int64_t ldh, int64_t n, const T* X, int64_t ldx, T* OUT,
                            int64_t ldo, int64_t ncols, T alpha, T beta, T gamma,
                            hipStream_t stream) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  const int tiles_m = static_cast<int>((n + BMC - 1) / BMC);
  const int tiles_n = static_cast<int>((ncols + BNC - 1) / BNC);
  const int64_t blocks = static_cast<int64_t>(tiles_m) * tiles_n;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hemm_step_kernel<T>, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0,
                     stream, H, ldh, static_cast<int>(n), X, ldx, OUT, ldo,
                     static_cast<int>(ncols), alpha, beta, gamma, tiles_m);
  return hipGetLastError();
}

template hipError_t launch_hemm_step<double>(const double*, int64_t, int64_t, const double*,
                                             int64_t, double*, int64_t, int64_t, double, double,
                                             double, hipStream_t);
template hipError_t launch_hemm_step<float>(const float*, int64_t, int64_t, const float*, int64_t,
                                            float*, int64_t, int64_t, float, float, float,
                                            hipStream_t);

static unsigned convert_blocks(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

hipError_t launch_convert_c128_to_c64(const double* src, int64_t lds, float* dst, int64_t ldd,
                                      int64_t rows, int64_t cols, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL((convert_kernel<double, float>), dim3(convert_blocks(rows * cols)), dim3(256),
                     0, stream, src, lds, dst, ldd, rows, cols);
  return hipGetLastError();
}

hipError_t launch_convert_c64_to_c128(const float* src, int64_t lds, double* dst, int64_t ldd,
                                      int64_t rows, int64_t cols, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL((convert_kernel<float, double>), dim3(convert_blocks(rows * cols)), dim3(256),
                     0, stream, src, lds, dst, ldd, rows, cols);
  return hipGetLastError();
}

}  // namespace chase
