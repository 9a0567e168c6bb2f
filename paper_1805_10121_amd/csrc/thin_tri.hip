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
// twice the scratch, about n^2 ncols / (4 S) bytes: with the super-tile edges S chosen below
// (8 for 1-2 columns, 4 for 3-5, 2 for 6-8 at large n) 1 to 13 per cent of the bytes of H.

#include <cmath>

#include "internal.h"

namespace chase {
namespace {

constexpr int kTB = 64;               // tile rows and columns (complex elements)
constexpr int kPitch = kTB + 1;       // LDS row pitch of a staged tile (complex elements)
constexpr int kTriThreads = 256;     // the fixup kernel's workgroup

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

// Super-tile edge for NC columns: the largest of 8, 4, 2 tiles with S * NC <= 20 (the row sums
// a thread keeps) that still leaves two workgroups per CU of a 256-CU device, else 1.
int tri_super(int64_t n, int nc) {
  const int64_t nb = (n + kTB - 1) / kTB;
  for (int S : {8, 4, 2}) {
    if (S * nc > 20) continue;
    const int64_t ns = (nb + S - 1) / S;
    if (ns * (ns + 1) / 2 >= 512) return S;
  }
  return 1;
}

// Thread roles: lane = row r of a tile (row product) or column k (column product); wave g of the
// four takes the quarter [16 g, 16 g + 16) of the summation index (k in the row product, r in the
// column product) for every column of X, so each element of H is read from LDS twice per tile
// whatever the number of columns.  The x value a step multiplies is the same for all lanes of a
// wave, so X is read with scalar loads into SGPRs: an LDS broadcast would still deliver 16 bytes
// to each of the 64 lanes, NC times the LDS traffic of H.  The waves' partial sums are added in
// LDS, in wave order.  LDS holds one tile (66.5 KB): two workgroups per CU.
constexpr int kTriWaves = 4;

template <int NC, int S>
__global__ __launch_bounds__(64 * kTriWaves, 2) void hemm_tri_kernel(
    const double* __restrict__ H, int64_t ldh, int n, const double* __restrict__ X, int64_t ldx,
    double2* __restrict__ part) {
  constexpr int NW = kTriWaves, NT = 64 * NW;
  constexpr int LOADS = kTB * kTB / NT;              // elements of a tile of H per thread
  constexpr int SS = S * S;
  constexpr int KQ = kTB / NW;                       // summation indices per wave
  constexpr int RS = kTB * kPitch / (NW * kTB * NC); // row blocks per reduction round
  constexpr int UNR = NC <= 3 ? 4 : 2;               // steps whose x loads are in flight together
  static_assert(S * NC <= 20 && RS >= 1, "sums exceed the registers or the reduction area");
  __shared__ double2 Hs[kTB * kPitch];  // also the reduction area
  const int tid = threadIdx.x, lane = tid & 63;
  const int g = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index (uniform)
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
  // register prefetch of a tile of H
  double2 ph[LOADS];
  auto prefetch = [&](int s) {
    const int I = P * S + s % S, J = Q * S + s / S;
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      const int row = I * kTB + lane, col = J * kTB + g + NW * q;  // one 1 KB column per wave
      ph[q] = (row < n && col < n)
                  ? Hc[static_cast<int64_t>(row) + static_cast<int64_t>(col) * ldh]
                  : double2{0.0, 0.0};
    }
  };

  double2 yrow[S][NC];  // this wave's part of the row sums of the super-row's S row blocks
  double2 ycol[NC];     // this wave's part of the current column block's sums
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int c = 0; c < NC; ++c) yrow[i][c] = double2{0.0, 0.0};
#pragma unroll
  for (int c = 0; c < NC; ++c) ycol[c] = double2{0.0, 0.0};

  double2* red = Hs;
  double2* pc = part + tri_slot(t, 1, S, NC);
  int s = next_valid(0);
  if (s < SS) prefetch(s);
  while (s < SS) {
    const int jj = s / S, ii = s % S;
    const int I = P * S + ii, J = Q * S + jj;
    const bool diag = P == Q && ii == jj;
    __syncthreads();  // the previous tile's products and reductions are done with the LDS
#pragma unroll
    for (int q = 0; q < LOADS; ++q) Hs[(g + NW * q) * kPitch + lane] = ph[q];
    const int sn = next_valid(s + 1);
    __syncthreads();
    if (sn < SS) prefetch(sn);  // in flight during the products below
    // x rows past the end of H are clamped to the last row: the matching elements of H were
    // loaded as zeros
    // row product: row r = lane of block I over k in this wave's quarter (k <= r on the diagonal)
    double2 acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      acc[c] = yrow[0][c];
#pragma unroll
      for (int i = 1; i < S; ++i)
        if (i == ii) acc[c] = yrow[i][c];
    }
#pragma unroll UNR
    for (int kk = 0; kk < KQ; ++kk) {
      const int k = g * KQ + kk;
      double2 h = Hs[k * kPitch + lane];
      if (diag && k > lane) h = double2{0.0, 0.0};
      const double2* xr = Xc + min(J * kTB + k, n - 1);
#pragma unroll
      for (int c = 0; c < NC; ++c) cmac(acc[c], h, xr[static_cast<int64_t>(c) * ldx]);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (i == ii) yrow[i][c] = acc[c];
    // column product: column k = lane of block J over r in this wave's quarter (r > k on the
    // diagonal), with conj(H[r, k]) = H[k, r]
#pragma unroll UNR
    for (int rr = 0; rr < KQ; ++rr) {
      const int r = g * KQ + rr;
      double2 h = Hs[lane * kPitch + r];
      if (diag && r <= lane) h = double2{0.0, 0.0};
      const double2* xr = Xc + min(I * kTB + r, n - 1);
#pragma unroll
      for (int c = 0; c < NC; ++c) cmac_conj(ycol[c], h, xr[static_cast<int64_t>(c) * ldx]);
    }
    // after the last tile of a super-column the column block's sum is complete: add the waves'
    // parts in wave order
    if (sn >= SS || sn / S != jj) {
      __syncthreads();  // every wave is done reading Hs
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        red[(g * kTB + lane) * NC + c] = ycol[c];
        ycol[c] = double2{0.0, 0.0};
      }
      __syncthreads();
      for (int e = tid; e < kTB * NC; e += NT) {
        const int k = e / NC, c = e % NC;
        double2 v = red[k * NC + c];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
          const double2 u = red[(w * kTB + k) * NC + c];
          v.x += u.x;
          v.y += u.y;
        }
        pc[(static_cast<int64_t>(jj) * kTB + k) * NC + c] = v;
      }
    }
    s = sn;
  }
  // every row block of the super-row, the waves' parts added in wave order, RS blocks per
  // round (a block past the last one of H keeps zeros; a column block of H always has a valid
  // tile in each super-tile of its super-column, so all the column slots the fixup reads were
  // written above)
  double2* pr = part + tri_slot(t, 0, S, NC);
#pragma unroll
  for (int i0 = 0; i0 < S; i0 += RS) {
    __syncthreads();  // the LDS is free: products done, previous round summed
#pragma unroll
    for (int i = i0; i < i0 + RS && i < S; ++i)
#pragma unroll
      for (int c = 0; c < NC; ++c) red[(((i - i0) * NW + g) * kTB + lane) * NC + c] = yrow[i][c];
    __syncthreads();
    const int nblk = (S - i0 < RS ? S - i0 : RS);
    for (int e = tid; e < nblk * kTB * NC; e += NT) {
      const int i = e / (kTB * NC), r = (e / NC) % kTB, c = e % NC;
      double2 v = red[((i * NW) * kTB + r) * NC + c];
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        const double2 u = red[((i * NW + w) * kTB + r) * NC + c];
        v.x += u.x;
        v.y += u.y;
      }
      pr[(static_cast<int64_t>(i0 + i) * kTB + r) * NC + c] = v;
    }
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

template <int NC, int S>
hipError_t launch_tri_s(const double* H, int64_t ldh, int64_t n, const double* X, int64_t ldx,
                        double* OUT, int64_t ldo, double alpha, double beta, double gamma,
                        double2* part, hipStream_t stream) {
  const int nb = static_cast<int>((n + kTB - 1) / kTB);
  const int NS = (nb + S - 1) / S;
  const int64_t tiles = static_cast<int64_t>(NS) * (NS + 1) / 2;
  hipLaunchKernelGGL((hemm_tri_kernel<NC, S>), dim3(static_cast<unsigned>(tiles)),
                     dim3(64 * kTriWaves), 0, stream, H, ldh, static_cast<int>(n), X, ldx, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((hemm_tri_fixup_kernel<S>), dim3(static_cast<unsigned>(nb)),
                     dim3(kTriThreads), 0, stream, X, ldx, OUT, ldo, static_cast<int>(n), NC, NS,
                     part, alpha, beta, gamma);
  return hipGetLastError();
}

template <int NC>
hipError_t launch_tri_c(const double* H, int64_t ldh, int64_t n, const double* X, int64_t ldx,
                        double* OUT, int64_t ldo, double alpha, double beta, double gamma,
                        double2* part, hipStream_t stream) {
  const int S = tri_super(n, NC);
  if constexpr (8 * NC <= 20)
    if (S == 8)
      return launch_tri_s<NC, 8>(H, ldh, n, X, ldx, OUT, ldo, alpha, beta, gamma, part, stream);
  if constexpr (4 * NC <= 20)
    if (S == 4)
      return launch_tri_s<NC, 4>(H, ldh, n, X, ldx, OUT, ldo, alpha, beta, gamma, part, stream);
  if (S == 2)
    return launch_tri_s<NC, 2>(H, ldh, n, X, ldx, OUT, ldo, alpha, beta, gamma, part, stream);
  return launch_tri_s<NC, 1>(H, ldh, n, X, ldx, OUT, ldo, alpha, beta, gamma, part, stream);
}

}  // namespace

size_t tri_scratch_bytes(int64_t n, int64_t ncols) {
  if (n <= 0 || ncols <= 0) return 0;
  const int S = tri_super(n, static_cast<int>(ncols));
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
  switch (ncols) {
#define CHASE_TRI_CASE(c) \
  case c:                 \
    return launch_tri_c<c>(H, ldh, n, X, ldx, OUT, ldo, alpha, beta, gamma, part, stream);
    CHASE_TRI_CASE(1) CHASE_TRI_CASE(2) CHASE_TRI_CASE(3) CHASE_TRI_CASE(4)
    CHASE_TRI_CASE(5) CHASE_TRI_CASE(6) CHASE_TRI_CASE(7) CHASE_TRI_CASE(8)
#undef CHASE_TRI_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace chase
