// One-triangle product for thin blocks: OUT <- alpha H X + gamma X + beta OUT for complex128
// Hermitian H and at most 8 columns, reading only the lower triangle of H (the Hermitian
// product of Sec. 5.1.1, which touches one triangle of the matrix).
//
// With few columns the product is bound by the bytes of H it reads; a full read moves 16 n^2
// bytes, one triangle 8 n^2.  Every stored element H[r, k] (r >= k) of the lower triangle is
// used twice: for row block I of the result through H[r, k] x[k] and, off the diagonal, for row
// block J through conj(H[r, k]) x[r] (H[k, r] = conj(H[r, k])).
//
// Schedule.  H is cut into 64 x 64 tiles and the tiles into S x S super-tiles; one workgroup
// takes one super-tile (P, Q) of the lower triangle (P >= Q; on the diagonal only the tiles
// with I >= J).  Each tile passes once through LDS (padded rows, so both the row-wise and the
// column-wise reads are free of bank conflicts), the next tile being prefetched into registers
// meanwhile.  A workgroup keeps the row-block sums of its super-row and the column-block sum of
// the current super-column in registers and writes them to its own slots of the scratch: no
// atomics.  A second kernel adds, for every row block, the slots that touch it in a fixed
// order (super-columns, then super-rows, ascending) and applies the epilogue, so the result is
// bitwise reproducible.
//
// Traffic per product: 8 n^2 bytes of H (plus the diagonal tiles' upper halves), the blocks, and
// twice the scratch, n^2 ncols / (2 S) bytes, i.e. a few per cent of H for the S chosen below.

#include <cmath>

#include "internal.h"

namespace chase {
namespace {

constexpr int kTB = 64;               // tile rows and columns (complex elements)
constexpr int kPitch = kTB + 1;       // LDS row pitch of a staged tile (complex elements)
constexpr int kTriThreads = 256;
constexpr int kTriLoads = kTB * kTB / kTriThreads;  // complex elements per thread and tile

// Super-tile (P, Q), P >= Q, of workgroup t = P (P + 1) / 2 + Q.
__device__ __forceinline__ void tri_coords(int64_t t, int* P, int* Q) {
  int p = static_cast<int>((sqrt(8.0 * static_cast<double>(t) + 1.0) - 1.0) * 0.5);
  while (static_cast<int64_t>(p) * (p + 1) / 2 > t) --p;
  while (static_cast<int64_t>(p + 1) * (p + 2) / 2 <= t) ++p;
  *P = p;
  *Q = static_cast<int>(t - static_cast<int64_t>(p) * (p + 1) / 2);
}

__device__ __forceinline__ void cmac(double2& acc, double2 a, double2 b) {  // acc += a b
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ void cmac_conj(double2& acc, double2 a, double2 b) {  // acc += conj(a) b
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// Partial sums of super-tile t: the S row blocks of its super-row (slot 0) and the S column
// blocks of its super-column (slot 1), each S x 64 x ncols complex values, element (i, r, c) at
// (i * 64 + r) * ncols + c.
__device__ __forceinline__ int64_t tri_slot(int64_t t, int which, int S, int ncols) {
  return (t * 2 + which) * static_cast<int64_t>(S) * kTB * ncols;
}

// Thread roles: lane = row r of a tile (row product) or column k (column product); the four
// waves share out the columns of X: wave g takes columns g, g + 4 (NCT = CMAX / 4 of them).
template <int CMAX>
constexpr int tri_occupancy() { return CMAX <= 4 ? 2 : 1; }  // by LDS: 74.5 or 82.5 KB

template <int CMAX, int S>
__global__ __launch_bounds__(kTriThreads, tri_occupancy<CMAX>()) void hemm_tri_kernel(
    const double* __restrict__ H, int64_t ldh, int n, const double* __restrict__ X, int64_t ldx,
    int ncols, double2* __restrict__ part) {
  constexpr int NCT = (CMAX + 3) / 4;
  constexpr int XL = (kTB * CMAX + kTriThreads - 1) / kTriThreads;  // x elements per thread
  constexpr int SS = S * S;
  __shared__ double2 Hs[kTB * kPitch];
  __shared__ double2 xJ[kTB * CMAX];
  __shared__ double2 xI[kTB * CMAX];
  const int tid = threadIdx.x, lane = tid & 63, g = tid >> 6;
  const int nb = (n + kTB - 1) / kTB;
  const int64_t t = blockIdx.x;
  int P, Q;
  tri_coords(t, &P, &Q);
  const double2* Hc = reinterpret_cast<const double2*>(H);
  const double2* Xc = reinterpret_cast<const double2*>(X);

  // the tiles of this super-tile in processing order: super-column block jj outer, row block
  // ii inner; on the diagonal super-tile only ii >= jj
  auto valid = [&](int s) {
    const int jj = s / S, ii = s % S;
    const int I = P * S + ii, J = Q * S + jj;
    return I < nb && J < nb && (P != Q || ii >= jj);
  };
  auto next_valid = [&](int s) {
    while (s < SS && !valid(s)) ++s;
    return s;
  };
  // register prefetch of a tile of H and the two blocks of X it meets
  double2 ph[kTriLoads], pxi[XL], pxj[XL];
  auto load_x = [&](double2 (&dst)[XL], int blk) {
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      const int e = tid + q * kTriThreads;
      const int r = e / CMAX, c = e % CMAX;
      const int row = blk * kTB + r;
      dst[q] = (e < kTB * CMAX && c < ncols && row < n)
                   ? Xc[static_cast<int64_t>(row) + static_cast<int64_t>(c) * ldx]
                   : double2{0.0, 0.0};
    }
  };
  auto prefetch = [&](int s) {
    const int I = P * S + s % S, J = Q * S + s / S;
#pragma unroll
    for (int q = 0; q < kTriLoads; ++q) {
      const int row = I * kTB + lane, col = J * kTB + g + 4 * q;  // one 1 KB column per wave
      ph[q] = (row < n && col < n)
                  ? Hc[static_cast<int64_t>(row) + static_cast<int64_t>(col) * ldh]
                  : double2{0.0, 0.0};
    }
    load_x(pxi, I);
    load_x(pxj, J);
  };

  double2 yrow[S][NCT];
  double2 ycol[NCT];
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int c = 0; c < NCT; ++c) yrow[i][c] = double2{0.0, 0.0};
#pragma unroll
  for (int c = 0; c < NCT; ++c) ycol[c] = double2{0.0, 0.0};

  double2* pc = part + tri_slot(t, 1, S, ncols);
  int s = next_valid(0);
  if (s < SS) prefetch(s);
  while (s < SS) {
    const int jj = s / S, ii = s % S;
    const bool diag = P == Q && ii == jj;
    __syncthreads();  // the previous tile's products are done with Hs, xI and xJ
#pragma unroll
    for (int q = 0; q < kTriLoads; ++q) Hs[(g + 4 * q) * kPitch + lane] = ph[q];
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      const int e = tid + q * kTriThreads;
      if (e < kTB * CMAX) {
        xI[e] = pxi[q];
        xJ[e] = pxj[q];
      }
    }
    const int sn = next_valid(s + 1);
    __syncthreads();
    if (sn < SS) prefetch(sn);  // in flight during the products below
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int col = g + 4 * c;
      if (col >= ncols) continue;
      // row product: row r = lane of block I over the tile's columns k (k <= r on the diagonal)
      double2 acc = yrow[0][c];
#pragma unroll
      for (int i = 1; i < S; ++i)
        if (i == ii) acc = yrow[i][c];
      const int kmax = diag ? lane + 1 : kTB;
      for (int k = 0; k < kmax; ++k) cmac(acc, Hs[k * kPitch + lane], xJ[k * CMAX + col]);
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (i == ii) yrow[i][c] = acc;
      // column product: column k = lane of block J over the tile's rows r (r > k on the
      // diagonal), with conj(H[r, k]) = H[k, r]
      double2 a2 = ycol[c];
      for (int r = diag ? lane + 1 : 0; r < kTB; ++r)
        cmac_conj(a2, Hs[lane * kPitch + r], xI[r * CMAX + col]);
      ycol[c] = a2;
    }
    // after the last tile of a super-column the column block's sum is complete
    if (sn >= SS || sn / S != jj) {
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        const int col = g + 4 * c;
        if (col < ncols) pc[(static_cast<int64_t>(jj) * kTB + lane) * ncols + col] = ycol[c];
        ycol[c] = double2{0.0, 0.0};
      }
    }
    s = sn;
  }
  // every row block of the super-row (a block past the last one of H keeps zeros; a column
  // block of H always has a valid tile in each super-tile of its super-column, so all the
  // column slots the fixup reads were written above)
  double2* pr = part + tri_slot(t, 0, S, ncols);
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int col = g + 4 * c;
      if (col < ncols) pr[(static_cast<int64_t>(i) * kTB + lane) * ncols + col] = yrow[i][c];
    }
}

// Row block b = blockIdx.x: y = sum over super-columns Q <= p of slot 0 of (p, Q), then over
// super-rows P >= p of slot 1 of (P, p) (p = b / S), in that order; then the epilogue.
template <int S>
__global__ __launch_bounds__(kTriThreads) void hemm_tri_fixup_kernel(
    const double* __restrict__ X, int64_t ldx, double* __restrict__ OUT, int64_t ldo, int n,
    int ncols, int NS, const double2* __restrict__ part, double alpha, double beta,
    double gamma) {
  const int b = blockIdx.x;
  const int p = b / S, i = b % S;
  for (int e = threadIdx.x; e < kTB * ncols; e += kTriThreads) {
    const int r = e / ncols, c = e % ncols;
    const int row = b * kTB + r;
    if (row >= n) continue;
    const int64_t off = (static_cast<int64_t>(i) * kTB + r) * ncols + c;
    double2 y{0.0, 0.0};
    for (int q = 0; q <= p; ++q) {
      const double2 v = part[tri_slot(static_cast<int64_t>(p) * (p + 1) / 2 + q, 0, S, ncols) + off];
      y.x += v.x;
      y.y += v.y;
    }
    for (int P = p; P < NS; ++P) {
      const double2 v = part[tri_slot(static_cast<int64_t>(P) * (P + 1) / 2 + p, 1, S, ncols) + off];
      y.x += v.x;
      y.y += v.y;
    }
    const double2 x = reinterpret_cast<const double2*>(X)[static_cast<int64_t>(row) +
                                                          static_cast<int64_t>(c) * ldx];
    double2* o = reinterpret_cast<double2*>(OUT) + static_cast<int64_t>(row) +
                 static_cast<int64_t>(c) * ldo;
    double2 res{alpha * y.x + gamma * x.x, alpha * y.y + gamma * x.y};
    if (beta != 0.0) {
      const double2 old = *o;
      res.x += beta * old.x;
      res.y += beta * old.y;
    }
    *o = res;
  }
}

// Super-tile edge: the largest of 8, 4, 2 tiles that still leaves two workgroups per CU of a
// 256-CU device, else 1.
int tri_super(int64_t n) {
  const int64_t nb = (n + kTB - 1) / kTB;
  for (int S : {8, 4, 2}) {
    const int64_t ns = (nb + S - 1) / S;
    if (ns * (ns + 1) / 2 >= 512) return S;
  }
  return 1;
}

template <int CMAX, int S>
hipError_t launch_tri_s(const double* H, int64_t ldh, int64_t n, const double* X, int64_t ldx,
                        double* OUT, int64_t ldo, int64_t ncols, double alpha, double beta,
                        double gamma, double2* part, hipStream_t stream) {
  const int nb = static_cast<int>((n + kTB - 1) / kTB);
  const int NS = (nb + S - 1) / S;
  const int64_t tiles = static_cast<int64_t>(NS) * (NS + 1) / 2;
  hipLaunchKernelGGL((hemm_tri_kernel<CMAX, S>), dim3(static_cast<unsigned>(tiles)),
                     dim3(kTriThreads), 0, stream, H, ldh, static_cast<int>(n), X, ldx,
                     static_cast<int>(ncols), part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((hemm_tri_fixup_kernel<S>), dim3(static_cast<unsigned>(nb)),
                     dim3(kTriThreads), 0, stream, X, ldx, OUT, ldo, static_cast<int>(n),
                     static_cast<int>(ncols), NS, part, alpha, beta, gamma);
  return hipGetLastError();
}

template <int CMAX>
hipError_t launch_tri_c(const double* H, int64_t ldh, int64_t n, const double* X, int64_t ldx,
                        double* OUT, int64_t ldo, int64_t ncols, double alpha, double beta,
                        double gamma, double2* part, hipStream_t stream) {
  switch (tri_super(n)) {
    case 8:
      return launch_tri_s<CMAX, 8>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, part, stream);
    case 4:
      return launch_tri_s<CMAX, 4>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, part, stream);
    case 2:
      return launch_tri_s<CMAX, 2>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, part, stream);
    default:
      return launch_tri_s<CMAX, 1>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, part, stream);
  }
}

}  // namespace

size_t tri_scratch_bytes(int64_t n, int64_t ncols) {
  if (n <= 0 || ncols <= 0) return 0;
  const int S = tri_super(n);
  const int64_t nb = (n + kTB - 1) / kTB;
  const int64_t NS = (nb + S - 1) / S;
  return static_cast<size_t>(NS * (NS + 1) / 2) * 2 * S * kTB * ncols * sizeof(double2);
}

hipError_t launch_hemm_tri(const double* H, int64_t ldh, int64_t n, const double* X, int64_t ldx,
                           double* OUT, int64_t ldo, int64_t ncols, double alpha, double beta,
                           double gamma, const ProductScratch& ps, hipStream_t stream) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  if (ncols > kTriMaxCols || n > 0x7fffffff) return hipErrorInvalidValue;
  const size_t need = tri_scratch_bytes(n, ncols);
  if (ps.sk_need) {
    *ps.sk_need = std::max(*ps.sk_need, need);
    return hipSuccess;
  }
  if (!ps.ptr || need > ps.bytes) return hipErrorInvalidValue;
  double2* part = static_cast<double2*>(ps.ptr);
  if (ncols <= 2)
    return launch_tri_c<2>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, part, stream);
  if (ncols <= 4)
    return launch_tri_c<4>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, part, stream);
  return launch_tri_c<8>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, part, stream);
}

}  // namespace chase
