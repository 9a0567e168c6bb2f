// Chebyshev-filter product kernels for gfx950 (CDNA4).
//
// One launch computes, for the active columns of the block (the steps of Alg. 4, Eq. (7)),
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
// Tiling: 256 threads (4 waves of 64) own a BMC x BNC complex output tile; each wave owns a
// sub-tile of 16x16 MFMA tiles.  K advances KT at a time through a double-buffered LDS stage
// fed by a register prefetch of the next stage.
//
// MFMA lane layouts used (16x16x4, checked on gfx950): A operand lane l holds A[l%16][l/16],
// B operand lane l holds B[l/16][l%16].  The accumulator's register r of lane l holds column
// l%16 and row (l/16) + 4r for f64, row 4(l/16) + r for f32.  The A-row permutation below makes
// registers (2p, 2p+1) of a lane the (Re, Im) rows of one complex row for both types, so the
// complex epilogue is lane local.

#include "internal.h"

#include <algorithm>
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

// Workgroup tile: BMC complex rows x BNC complex columns, K staged KT at a time; the four
// waves form a WR x WC grid, each owning (BMC/WR) x (BNC/WC) complex outputs, i.e. RT row
// slabs of 8 complex (16 real) rows times CG column groups of 16, each group an (Re X, Im X)
// pair of MFMA tiles.
// PROMOTE_ > 0 (complex64 only): every PROMOTE_ K stages the FP32 MFMA accumulators are added
// into FP64 accumulators and cleared, so rounding error stops growing with the length of the
// dot product (FP32 products, FP64 sums across stages).
// BKT_ (B k-major): the B stage is stored one real column per LDS row, KT + 1 values apart, so
// both the staging stores (consecutive k) and the MFMA operand reads (16 columns at one k) fall
// in distinct banks; otherwise it is stored one k per row, 2 BNC + PAD_ values apart.
// PADB_ < 0: the B stage rows use the A padding PAD_.
// SCHED_ > 0: the LDS stores of the next stage are interleaved with the MFMAs of the last K step
// of the current one (instead of following them); SCHED_ > 1 also interleaves the next stage's
// global loads with the MFMAs of the first K step.
template <typename T, int BMC_, int BNC_, int KT_, int WR_, int WC_, int PAD_ = 2, int PROMOTE_ = 0,
          bool BKT_ = false, int PADB_ = -1, int SCHED_ = 0>
struct Tile {
  static constexpr int KIND = 0;  // 4M real embedding of interleaved complex H
  static constexpr int OCC = 2;   // workgroups per CU the tile is built for
  static constexpr int BMC = BMC_, BNC = BNC_, KT = KT_, WR = WR_, WC = WC_;
  static constexpr int PROMOTE = PROMOTE_;
  static constexpr int SCHED = SCHED_;
  static constexpr bool BKT = BKT_;
  static constexpr int RT = BMC / WR / 8;
  static constexpr int CG = BNC / WC / 16;
  static constexpr int AR = 2 * BMC + PAD_;  // padded real rows per A stage row (k fixed)
  static constexpr int BR = 2 * BNC + (PADB_ < 0 ? PAD_ : PADB_);  // padded real columns per B stage row
  static constexpr int BK = KT + 1;          // padded k per B stage column (BKT_ layout)
  static constexpr int A_PER = BMC * KT / kThreads;
  static constexpr int B_PER = BNC * KT / kThreads;
  static_assert(WR * WC == 4, "four waves");
  static_assert(RT >= 1 && CG >= 1, "wave tile too small");
  static_assert(A_PER * kThreads == BMC * KT && B_PER * kThreads == BNC * KT, "load split");
  using acc_t = typename Acc<T>::type;
  using v2 = typename Acc<T>::v2;
  struct SmemK {
    T As[2][KT][AR];
    T Bs[2][KT][BR];
  };
  struct SmemT {
    T As[2][KT][AR];
    T Bs[2][2 * BNC][BK];
  };
  using Smem = typename std::conditional<BKT_, SmemT, SmemK>::type;
  struct Frag64 {
    acc_t acc[RT][CG][2];
    double acc64[RT][CG][2][4];
  };
  struct Frag32 {
    acc_t acc[RT][CG][2];
  };
  using Frag = typename std::conditional<(PROMOTE_ > 0), Frag64, Frag32>::type;
};

// acc <- R[i0.., k] [Re X | Im X][k, j0..] summed over the K stages ka <= kt < kb.
// V16 (complex64 only): global loads of two consecutive complex elements (16 bytes); the caller
// guarantees 16-byte aligned H and X and even leading dimensions.
template <typename T, class C, bool V16 = false>
__device__ __forceinline__ void tile_mainloop_4m(typename C::Smem& sm, typename C::Frag& f,
                                              const T* __restrict__ H, int64_t ldh, int n,
                                              const T* __restrict__ X, int64_t ldx, int ncols,
                                              int i0, int j0, int ka, int kb) {
  using v2 = typename C::v2;
  using acc_t = typename C::acc_t;
  constexpr int VEC = (V16 && sizeof(T) == 4) ? 2 : 1;  // complex elements per global load
  // exactly VEC elements: alignment = size, so a copy never touches a neighbour
  struct alignas(sizeof(v2) * VEC) VL { v2 e[VEC]; };
  static_assert(sizeof(VL) == sizeof(v2) * VEC, "load unit size");
  constexpr int A_LD = C::BMC * C::KT / (kThreads * VEC);
  constexpr int B_LD = C::BNC * C::KT / (kThreads * VEC);
  static_assert(A_LD * kThreads * VEC == C::BMC * C::KT, "A load split");
  static_assert(B_LD * kThreads * VEC == C::BNC * C::KT, "B load split");
  static_assert(VEC == 1 || (C::AR * sizeof(T)) % 16 == 0, "16-byte LDS rows for V16");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int wr = wave / C::WC, wc = wave % C::WC;
  VL ra[A_LD], rb[B_LD];

  // Load q of a thread is load 0 moved by a whole number of H columns (A) or X columns (B): one
  // base pointer per operand plus uniform offsets.  Every load is issued unconditionally (a unit
  // that is not wholly inside the operand reads from the operand's first element instead) and is
  // zeroed when the stage is written to LDS, after the wait that the LDS store needs anyway, so
  // no load is followed by an early wait.  Two-element units need n even (the launcher's rule),
  // so a unit is either wholly inside the operand or wholly outside.
  static_assert(kThreads % (C::BMC / VEC) == 0 && kThreads % (C::KT / VEC) == 0, "load strides");
  static_assert(A_LD + B_LD <= 32, "validity bits");
  const bool tile_full = i0 + C::BMC <= n && j0 + C::BNC <= ncols;
  const T* const pa0 = H + 2 * (static_cast<int64_t>(i0 + (tid % (C::BMC / VEC)) * VEC) +
                                static_cast<int64_t>(tid / (C::BMC / VEC)) * ldh);
  const T* const pb0 = X + 2 * (static_cast<int64_t>((tid % (C::KT / VEC)) * VEC) +
                                static_cast<int64_t>(j0 + tid / (C::KT / VEC)) * ldx);
  const int64_t sa = 2 * static_cast<int64_t>(kThreads / (C::BMC / VEC)) * ldh;
  const int64_t sb = 2 * static_cast<int64_t>(kThreads / (C::KT / VEC)) * ldx;
  uint32_t valid = 0;  // bit u: load u (A loads, then B loads) is inside its operand

  auto load_tiles = [&](int k0) {
    const bool fast = tile_full && k0 + C::KT <= n;
    const T* a = pa0 + 2 * static_cast<int64_t>(k0) * ldh;
    const T* b = pb0 + 2 * static_cast<int64_t>(k0);
    uint32_t bits = 0;
#pragma unroll
    for (int q = 0; q < A_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int kk = idx / (C::BMC / VEC), ci = (idx % (C::BMC / VEC)) * VEC;
      const bool ok = fast || (k0 + kk < n && i0 + ci + VEC - 1 < n);
      ra[q] = *reinterpret_cast<const VL*>(ok ? a + q * sa : H);
      bits |= (ok ? 1u : 0u) << q;
    }
#pragma unroll
    for (int q = 0; q < B_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int jj = idx / (C::KT / VEC), kk = (idx % (C::KT / VEC)) * VEC;
      const bool ok = fast || (j0 + jj < ncols && k0 + kk + VEC - 1 < n);
      rb[q] = *reinterpret_cast<const VL*>(ok ? b + q * sb : X);
      bits |= (ok ? 1u : 0u) << (A_LD + q);
    }
    valid = bits;
  };
  // The unit as it goes to LDS: zero when it lies outside the operand.
  auto fix_unit = [&](VL v, int u) {
    if (!((valid >> u) & 1u)) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) v.e[e] = v2{T(0), T(0)};
    }
    return v;
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int q = 0; q < A_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int kk = idx / (C::BMC / VEC), ci = (idx % (C::BMC / VEC)) * VEC;
      *reinterpret_cast<VL*>(&sm.As[buf][kk][2 * ci]) = fix_unit(ra[q], q);
    }
#pragma unroll
    for (int q = 0; q < B_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int jj = idx / (C::KT / VEC), kk = (idx % (C::KT / VEC)) * VEC;
      const VL v = fix_unit(rb[q], A_LD + q);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        if constexpr (C::BKT) {
          sm.Bs[buf][jj][kk + e] = v.e[e].x;
          sm.Bs[buf][C::BNC + jj][kk + e] = v.e[e].y;
        } else {
          sm.Bs[buf][kk + e][jj] = v.e[e].x;
          sm.Bs[buf][kk + e][C::BNC + jj] = v.e[e].y;
        }
      }
    }
  };

#pragma unroll
  for (int a = 0; a < C::RT; ++a)
#pragma unroll
    for (int b = 0; b < C::CG; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        f.acc[a][b][c] = acc_t{0};
        if constexpr (C::PROMOTE > 0) {
#pragma unroll
          for (int e = 0; e < 4; ++e) f.acc64[a][b][c][e] = 0.0;
        }
      }

  const int arow = a_row<T>(li);
  const int rbase = wr * (C::BMC / C::WR) * 2;  // first real row of this wave in the A stage
  const int cbase = wc * (C::BNC / C::WC);      // first complex column of this wave
  load_tiles(ka * C::KT);
  store_tiles(0);
  __syncthreads();
  // Operand fragments of K step s (4 values of k) from LDS buffer cur.
  auto fragments = [&](int cur, int s, T (&a)[C::RT], T (&b)[C::CG][2]) {
    const int k = 4 * s + g;
#pragma unroll
    for (int rt = 0; rt < C::RT; ++rt) a[rt] = sm.As[cur][k][rbase + rt * 16 + arow];
#pragma unroll
    for (int cg = 0; cg < C::CG; ++cg) {
      if constexpr (C::BKT) {
        b[cg][0] = sm.Bs[cur][cbase + cg * 16 + li][k];
        b[cg][1] = sm.Bs[cur][C::BNC + cbase + cg * 16 + li][k];
      } else {
        b[cg][0] = sm.Bs[cur][k][cbase + cg * 16 + li];
        b[cg][1] = sm.Bs[cur][k][C::BNC + cbase + cg * 16 + li];
      }
    }
  };
  auto products = [&](const T (&a)[C::RT], const T (&b)[C::CG][2]) {
#pragma unroll
    for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
      for (int cg = 0; cg < C::CG; ++cg)
#pragma unroll
        for (int p = 0; p < 2; ++p) f.acc[rt][cg][p] = mfma(a[rt], b[cg][p], f.acc[rt][cg][p]);
  };
  auto promote = [&](int kt) {
    if constexpr (C::PROMOTE > 0) {
      if ((kt - ka + 1) % C::PROMOTE == 0 || kt + 1 == kb) {
#pragma unroll
        for (int a = 0; a < C::RT; ++a)
#pragma unroll
          for (int b = 0; b < C::CG; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
#pragma unroll
              for (int e = 0; e < 4; ++e) f.acc64[a][b][c][e] += static_cast<double>(f.acc[a][b][c][e]);
              f.acc[a][b][c] = acc_t{0};
            }
      }
    }
  };
  constexpr int STEPS = C::KT / 4;
  constexpr int NMFMA = C::RT * C::CG * 2;

  if constexpr (C::SCHED == 0) {
    for (int kt = ka; kt < kb; ++kt) {
      const int cur = (kt - ka) & 1;
      if (kt + 1 < kb) load_tiles((kt + 1) * C::KT);
#pragma unroll
      for (int s = 0; s < STEPS; ++s) {
        T a[C::RT], b[C::CG][2];
        fragments(cur, s, a, b);
        products(a, b);
      }
      promote(kt);
      if (kt + 1 < kb) store_tiles(cur ^ 1);
      __syncthreads();
    }
  } else {
    int kt = ka;
    for (; kt + 1 < kb; ++kt) {  // stages followed by another: prefetch and stage the next one
      const int cur = (kt - ka) & 1;
#pragma unroll
      for (int s = 0; s < STEPS; ++s) {
        T a[C::RT], b[C::CG][2];
        fragments(cur, s, a, b);
        if (s == 0) load_tiles((kt + 1) * C::KT);
        if (s == STEPS - 1) store_tiles(cur ^ 1);
        products(a, b);
        if (s == 0 && C::SCHED > 1) {
          constexpr int NL = A_LD + B_LD;
#pragma unroll
          for (int i = 0; i < NL; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, NMFMA / NL > 0 ? NMFMA / NL : 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
          }
        }
        if (s == STEPS - 1) {
          constexpr int NW = A_LD + B_LD;
#pragma unroll
          for (int i = 0; i < NW; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, NMFMA / NW > 0 ? NMFMA / NW : 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
          }
        }
      }
      promote(kt);
      __syncthreads();
    }
    if (kt < kb) {  // last stage
      const int cur = (kt - ka) & 1;
#pragma unroll
      for (int s = 0; s < STEPS; ++s) {
        T a[C::RT], b[C::CG][2];
        fragments(cur, s, a, b);
        products(a, b);
      }
      promote(kt);
      __syncthreads();
    }
  }
}

// Visit the complex results held by this lane: fn(row_in_tile, col_in_tile, re, im).
template <typename T, class C, typename Fn>
__device__ __forceinline__ void tile_foreach_4m(const typename C::Frag& f, Fn&& fn) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int wr = wave / C::WC, wc = wave % C::WC;
#pragma unroll
  for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
    for (int cg = 0; cg < C::CG; ++cg)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int r = wr * (C::BMC / C::WR) + rt * 8 + c_row<T>(g, p);
        const int c = wc * (C::BNC / C::WC) + cg * 16 + li;
        if constexpr (C::PROMOTE > 0) {
          const double hre = f.acc64[rt][cg][0][2 * p] - f.acc64[rt][cg][1][2 * p + 1];
          const double him = f.acc64[rt][cg][1][2 * p] + f.acc64[rt][cg][0][2 * p + 1];
          fn(r, c, static_cast<T>(hre), static_cast<T>(him));
        } else {
          const T hre = f.acc[rt][cg][0][2 * p] - f.acc[rt][cg][1][2 * p + 1];
          const T him = f.acc[rt][cg][1][2 * p] + f.acc[rt][cg][0][2 * p + 1];
          fn(r, c, hre, him);
        }
      }
}

// 3M complex product (H stored as two real planes: Re H, then Im H at an offset of ldh * n
// values), on FP32 MFMA for complex64 data or FP64 MFMA for complex128 data.  With
// T1 = ReH ReX, T2 = ImH ImX and T3 = (ReH + ImH)(ReX + ImX):  Re(HX) = T1 - T2,
// Im(HX) = T3 - T1 - T2 -- three real products (6 real flops per complex multiply-add) instead
// of four.  The sums ReH + ImH and ReX + ImX are formed in registers from the LDS planes.  Each
// wave owns RT x CG MFMA tiles of 16 x 16 complex outputs.
// PROMOTE_ > 0 (FP32): every PROMOTE_ K stages the three FP32 partial products are combined in
// FP32 into the real and imaginary parts of that stretch, T1 - T2 and T3 - T1 - T2, which are
// added into two FP64 sums and the FP32 accumulators cleared.  Keeping two FP64 sums instead of
// three saves 32 registers per lane, enough for three workgroups per CU.
// OCC_: workgroups per CU the tile is built for (launch bounds and the stream-K grid).
template <int BMC_, int BNC_, int KT_, int WR_, int WC_, int PAD_ = 4, int PROMOTE_ = 1,
          typename T_ = float, int OCC_ = 2>
struct Tile3M {
  using T = T_;  // float: complex64 data, FP32 MFMA; double: complex128 data, FP64 MFMA
  static constexpr int KIND = 1;
  static constexpr int OCC = OCC_;
  static constexpr int BMC = BMC_, BNC = BNC_, KT = KT_, WR = WR_, WC = WC_;
  static constexpr int PROMOTE = PROMOTE_;
  static constexpr int RT = BMC / WR / 16;
  static constexpr int CG = BNC / WC / 16;
  static constexpr int AR = BMC + PAD_;
  static constexpr int BR = BNC + PAD_;
  static_assert(WR * WC == 4 && RT >= 1 && CG >= 1, "wave grid");
  static_assert((AR * sizeof(T)) % 16 == 0, "16-byte LDS rows");
  static_assert(sizeof(T) == 4 || PROMOTE_ == 0, "promotion applies to FP32 accumulators");
  using acc_t = typename Acc<T>::type;
  using v2 = typename Acc<T>::v2;
  struct Smem {
    T Are[2][KT][AR];
    T Aim[2][KT][AR];
    T Bre[2][KT][BR];
    T Bim[2][KT][BR];
  };
  struct Frag64 {
    acc_t acc[RT][CG][3];
    double acc64[RT][CG][2][4];  // FP64 sums of the real and imaginary parts
  };
  struct Frag32 {
    acc_t acc[RT][CG][3];
  };
  using Frag = typename std::conditional<(PROMOTE_ > 0), Frag64, Frag32>::type;
};

template <class C, bool V16>
__device__ __forceinline__ void tile_mainloop_3m(typename C::Smem& sm, typename C::Frag& f,
                                                 const typename C::T* __restrict__ H, int64_t ldh,
                                                 int n, const typename C::T* __restrict__ X,
                                                 int64_t ldx, int ncols, int i0, int j0, int ka,
                                                 int kb) {
  using T = typename C::T;
  using acc_t = typename C::acc_t;
  using v2 = typename C::v2;
  // 16-byte global loads when V16: consecutive rows of one plane (4 floats or 2 doubles) and
  // one or two complex elements of X
  constexpr int AV = V16 ? 16 / static_cast<int>(sizeof(T)) : 1;
  constexpr int BV = V16 ? 8 / static_cast<int>(sizeof(T)) : 1;
  constexpr int A_LD = C::BMC * C::KT / (kThreads * AV);
  constexpr int B_LD = C::BNC * C::KT / (kThreads * BV);
  static_assert(A_LD * kThreads * AV == C::BMC * C::KT, "A split");
  static_assert(B_LD * kThreads * BV == C::BNC * C::KT, "B split");
  // exactly AV values / BV complex elements: alignment = size, so a copy never touches a
  // neighbour
  struct alignas(sizeof(T) * AV) AL { T e[AV]; };
  struct alignas(2 * sizeof(T) * BV) BL { v2 e[BV]; };
  static_assert(sizeof(AL) == sizeof(T) * AV && sizeof(BL) == 2 * sizeof(T) * BV,
                "load unit size");
  const T* __restrict__ Hi = H + ldh * static_cast<int64_t>(n);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int wr = wave / C::WC, wc = wave % C::WC;
  AL rar[A_LD], rai[A_LD];
  BL rb[B_LD];

  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int q = 0; q < A_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int kk = idx / (C::BMC / AV), ri = (idx % (C::BMC / AV)) * AV;
      const int row = i0 + ri, col = k0 + kk;
      const int64_t off = static_cast<int64_t>(row) + static_cast<int64_t>(col) * ldh;
      if (col < n && row + AV - 1 < n) {
        rar[q] = *reinterpret_cast<const AL*>(H + off);
        rai[q] = *reinterpret_cast<const AL*>(Hi + off);
      } else {
#pragma unroll
        for (int e = 0; e < AV; ++e) {
          const bool ok = col < n && row + e < n;
          rar[q].e[e] = ok ? H[off + e] : T(0);
          rai[q].e[e] = ok ? Hi[off + e] : T(0);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < B_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int jj = idx / (C::KT / BV), kk = (idx % (C::KT / BV)) * BV;
      const int row = k0 + kk, col = j0 + jj;
      const T* src = X + 2 * (static_cast<int64_t>(row) + static_cast<int64_t>(col) * ldx);
      if (col < ncols && row + BV - 1 < n) {
        rb[q] = *reinterpret_cast<const BL*>(src);
      } else {
#pragma unroll
        for (int e = 0; e < BV; ++e)
          rb[q].e[e] = (col < ncols && row + e < n) ? reinterpret_cast<const v2*>(src)[e]
                                                     : v2{T(0), T(0)};
      }
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int q = 0; q < A_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int kk = idx / (C::BMC / AV), ri = (idx % (C::BMC / AV)) * AV;
      *reinterpret_cast<AL*>(&sm.Are[buf][kk][ri]) = rar[q];
      *reinterpret_cast<AL*>(&sm.Aim[buf][kk][ri]) = rai[q];
    }
#pragma unroll
    for (int q = 0; q < B_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int jj = idx / (C::KT / BV), kk = (idx % (C::KT / BV)) * BV;
#pragma unroll
      for (int e = 0; e < BV; ++e) {
        sm.Bre[buf][kk + e][jj] = rb[q].e[e].x;
        sm.Bim[buf][kk + e][jj] = rb[q].e[e].y;
      }
    }
  };

#pragma unroll
  for (int a = 0; a < C::RT; ++a)
#pragma unroll
    for (int b = 0; b < C::CG; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        f.acc[a][b][c] = acc_t{0};
        if constexpr (C::PROMOTE > 0) {
          if (c < 2) {
#pragma unroll
            for (int e = 0; e < 4; ++e) f.acc64[a][b][c][e] = 0.0;
          }
        }
      }

  const int rbase = wr * (C::BMC / C::WR);
  const int cbase = wc * (C::BNC / C::WC);
  load_tiles(ka * C::KT);
  store_tiles(0);
  __syncthreads();
  for (int kt = ka; kt < kb; ++kt) {
    const int cur = (kt - ka) & 1;
    if (kt + 1 < kb) load_tiles((kt + 1) * C::KT);
#pragma unroll
    for (int s = 0; s < C::KT / 4; ++s) {
      const int k = 4 * s + g;
      T ar[C::RT], ai[C::RT], as[C::RT], br[C::CG], bi[C::CG], bs[C::CG];
#pragma unroll
      for (int rt = 0; rt < C::RT; ++rt) {
        ar[rt] = sm.Are[cur][k][rbase + rt * 16 + li];
        ai[rt] = sm.Aim[cur][k][rbase + rt * 16 + li];
        as[rt] = ar[rt] + ai[rt];
      }
#pragma unroll
      for (int cg = 0; cg < C::CG; ++cg) {
        br[cg] = sm.Bre[cur][k][cbase + cg * 16 + li];
        bi[cg] = sm.Bim[cur][k][cbase + cg * 16 + li];
        bs[cg] = br[cg] + bi[cg];
      }
#pragma unroll
      for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
        for (int cg = 0; cg < C::CG; ++cg) {
          f.acc[rt][cg][0] = mfma(ar[rt], br[cg], f.acc[rt][cg][0]);
          f.acc[rt][cg][1] = mfma(ai[rt], bi[cg], f.acc[rt][cg][1]);
          f.acc[rt][cg][2] = mfma(as[rt], bs[cg], f.acc[rt][cg][2]);
        }
    }
    if constexpr (C::PROMOTE > 0) {
      if ((kt - ka + 1) % C::PROMOTE == 0 || kt + 1 == kb) {
#pragma unroll
        for (int a = 0; a < C::RT; ++a)
#pragma unroll
          for (int b = 0; b < C::CG; ++b) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const T t1 = f.acc[a][b][0][e], t2 = f.acc[a][b][1][e], t3 = f.acc[a][b][2][e];
              f.acc64[a][b][0][e] += static_cast<double>(t1 - t2);
              f.acc64[a][b][1][e] += static_cast<double>(t3 - t1 - t2);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) f.acc[a][b][c] = acc_t{0};
          }
      }
    }
    if (kt + 1 < kb) store_tiles(cur ^ 1);
    __syncthreads();
  }
}

template <class C, typename Fn>
__device__ __forceinline__ void tile_foreach_3m(const typename C::Frag& f, Fn&& fn) {
  using T = typename C::T;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int wr = wave / C::WC, wc = wave % C::WC;
#pragma unroll
  for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
    for (int cg = 0; cg < C::CG; ++cg)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // accumulator row layout: FP64 MFMA rows g + 4r, FP32 MFMA rows 4g + r
        const int row = wr * (C::BMC / C::WR) + rt * 16 + (sizeof(T) == 8 ? g + 4 * r : 4 * g + r);
        const int col = wc * (C::BNC / C::WC) + cg * 16 + li;
        if constexpr (C::PROMOTE > 0) {
          fn(row, col, static_cast<float>(f.acc64[rt][cg][0][r]),
             static_cast<float>(f.acc64[rt][cg][1][r]));
        } else {
          const T t1 = f.acc[rt][cg][0][r], t2 = f.acc[rt][cg][1][r], t3 = f.acc[rt][cg][2][r];
          fn(row, col, t1 - t2, t3 - t1 - t2);
        }
      }
}

// ---------------------------------------------------------------------------------------------
// Real symmetric H (the real variants of the solver): the product is a plain real GEMM, so the
// MFMA operands are H and X themselves.  BM x BN real outputs per workgroup, K staged KT at a
// time as in the complex tiles; each wave owns RT x CT MFMA tiles of 16 x 16.
template <typename T, int BM_, int BN_, int KT_, int WR_, int WC_, int PAD_ = 2>
struct TileR {
  static constexpr int KIND = 2;
  static constexpr int OCC = 2;
  static constexpr int BMC = BM_, BNC = BN_, KT = KT_, WR = WR_, WC = WC_;  // real rows / columns
  static constexpr int PROMOTE = 0;
  static constexpr int RT = BM_ / WR_ / 16;
  static constexpr int CT = BN_ / WC_ / 16;
  static constexpr int AR = BM_ + PAD_;
  static constexpr int BR = BN_ + PAD_;
  static_assert(WR * WC == 4, "four waves");
  static_assert(RT >= 1 && CT >= 1, "wave tile too small");
  using acc_t = typename Acc<T>::type;
  struct Smem {
    T As[2][KT][AR];
    T Bs[2][KT][BR];
  };
  struct Frag {
    acc_t acc[RT][CT];
  };
};

// acc <- H[i0.., k] X[k, j0..] over the K stages ka <= kt < kb (real H and X, column-major).
// V2: loads of two consecutive elements (16 bytes for double); the caller guarantees aligned H
// and X and even n, ldh and ldx, so a two-element unit is wholly inside or wholly outside.
template <typename T, class C, bool V2 = false>
__device__ __forceinline__ void tile_mainloop_real(typename C::Smem& sm, typename C::Frag& f,
                                                const T* __restrict__ H, int64_t ldh, int n,
                                                const T* __restrict__ X, int64_t ldx, int ncols,
                                                int i0, int j0, int ka, int kb) {
  using acc_t = typename C::acc_t;
  // elements per global load of A and of B (B stays at one element when a stage of B has
  // fewer than two elements per thread)
  constexpr int VEA = V2 ? 2 : 1;
  constexpr int VEB = (V2 && C::BNC * C::KT >= 2 * kThreads) ? 2 : 1;
  struct alignas(sizeof(T) * VEA) VLA { T e[VEA]; };
  struct alignas(sizeof(T) * VEB) VLB { T e[VEB]; };
  static_assert(sizeof(VLA) == sizeof(T) * VEA && sizeof(VLB) == sizeof(T) * VEB, "unit size");
  constexpr int A_LD = C::BMC * C::KT / (kThreads * VEA);
  constexpr int B_LD = C::BNC * C::KT / (kThreads * VEB);
  static_assert(A_LD >= 1 && A_LD * kThreads * VEA == C::BMC * C::KT, "A load split");
  static_assert(B_LD >= 1 && B_LD * kThreads * VEB == C::BNC * C::KT, "B load split");
  static_assert(kThreads % (C::BMC / VEA) == 0 && kThreads % (C::KT / VEB) == 0, "load strides");
  static_assert(VEA == 1 || (C::AR * sizeof(T)) % (sizeof(T) * VEA) == 0, "aligned LDS rows");
  static_assert(A_LD + B_LD <= 32, "validity bits");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int wr = wave / C::WC, wc = wave % C::WC;
  VLA ra[A_LD];
  VLB rb[B_LD];
  // Same load scheme as the complex tiles: one base pointer per operand, unconditional loads,
  // out-of-range units zeroed when written to LDS.
  const bool tile_full = i0 + C::BMC <= n && j0 + C::BNC <= ncols;
  const T* const pa0 = H + static_cast<int64_t>(i0 + (tid % (C::BMC / VEA)) * VEA) +
                       static_cast<int64_t>(tid / (C::BMC / VEA)) * ldh;
  const T* const pb0 = X + static_cast<int64_t>((tid % (C::KT / VEB)) * VEB) +
                       static_cast<int64_t>(j0 + tid / (C::KT / VEB)) * ldx;
  const int64_t sa = static_cast<int64_t>(kThreads / (C::BMC / VEA)) * ldh;
  const int64_t sb = static_cast<int64_t>(kThreads / (C::KT / VEB)) * ldx;
  uint32_t valid = 0;
  auto load_tiles = [&](int k0) {
    const bool fast = tile_full && k0 + C::KT <= n;
    const T* a = pa0 + static_cast<int64_t>(k0) * ldh;
    const T* b = pb0 + static_cast<int64_t>(k0);
    uint32_t bits = 0;
#pragma unroll
    for (int q = 0; q < A_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int kk = idx / (C::BMC / VEA), ci = (idx % (C::BMC / VEA)) * VEA;
      const bool ok = fast || (k0 + kk < n && i0 + ci + VEA - 1 < n);
      ra[q] = *reinterpret_cast<const VLA*>(ok ? a + q * sa : H);
      bits |= (ok ? 1u : 0u) << q;
    }
#pragma unroll
    for (int q = 0; q < B_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int jj = idx / (C::KT / VEB), kk = (idx % (C::KT / VEB)) * VEB;
      const bool ok = fast || (j0 + jj < ncols && k0 + kk + VEB - 1 < n);
      rb[q] = *reinterpret_cast<const VLB*>(ok ? b + q * sb : X);
      bits |= (ok ? 1u : 0u) << (A_LD + q);
    }
    valid = bits;
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int q = 0; q < A_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int kk = idx / (C::BMC / VEA), ci = (idx % (C::BMC / VEA)) * VEA;
      VLA v = ra[q];
      if (!((valid >> q) & 1u)) {
#pragma unroll
        for (int e = 0; e < VEA; ++e) v.e[e] = T(0);
      }
      *reinterpret_cast<VLA*>(&sm.As[buf][kk][ci]) = v;
    }
#pragma unroll
    for (int q = 0; q < B_LD; ++q) {
      const int idx = tid + kThreads * q;
      const int jj = idx / (C::KT / VEB), kk = (idx % (C::KT / VEB)) * VEB;
      const bool ok = (valid >> (A_LD + q)) & 1u;
#pragma unroll
      for (int e = 0; e < VEB; ++e) sm.Bs[buf][kk + e][jj] = ok ? rb[q].e[e] : T(0);
    }
  };

#pragma unroll
  for (int a = 0; a < C::RT; ++a)
#pragma unroll
    for (int b = 0; b < C::CT; ++b) f.acc[a][b] = acc_t{0};

  const int rbase = wr * (C::BMC / C::WR);
  const int cbase = wc * (C::BNC / C::WC);
  load_tiles(ka * C::KT);
  store_tiles(0);
  __syncthreads();
  for (int kt = ka; kt < kb; ++kt) {
    const int cur = (kt - ka) & 1;
    if (kt + 1 < kb) load_tiles((kt + 1) * C::KT);
#pragma unroll
    for (int s = 0; s < C::KT / 4; ++s) {
      const int k = 4 * s + g;
      T a[C::RT], b[C::CT];
#pragma unroll
      for (int rt = 0; rt < C::RT; ++rt) a[rt] = sm.As[cur][k][rbase + rt * 16 + li];
#pragma unroll
      for (int ct = 0; ct < C::CT; ++ct) b[ct] = sm.Bs[cur][k][cbase + ct * 16 + li];
#pragma unroll
      for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < C::CT; ++ct) f.acc[rt][ct] = mfma(a[rt], b[ct], f.acc[rt][ct]);
    }
    if (kt + 1 < kb) store_tiles(cur ^ 1);
    __syncthreads();
  }
}

// Visit the real results held by this lane: fn(row_in_tile, col_in_tile, value, 0).
template <typename T, class C, typename Fn>
__device__ __forceinline__ void tile_foreach_real(const typename C::Frag& f, Fn&& fn) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int wr = wave / C::WC, wc = wave % C::WC;
#pragma unroll
  for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < C::CT; ++ct)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = sizeof(T) == 8 ? g + 4 * e : 4 * g + e;  // accumulator row layout
        fn(wr * (C::BMC / C::WR) + rt * 16 + rr, wc * (C::BNC / C::WC) + ct * 16 + li,
           static_cast<T>(f.acc[rt][ct][e]), T(0));
      }
}

// Dispatch on the tile kind (4M interleaved or 3M planar).
template <typename T, class C, bool V16 = false>
__device__ __forceinline__ void tile_mainloop(typename C::Smem& sm, typename C::Frag& f,
                                              const T* __restrict__ H, int64_t ldh, int n,
                                              const T* __restrict__ X, int64_t ldx, int ncols,
                                              int i0, int j0, int ka, int kb) {
  if constexpr (C::KIND == 1)
    tile_mainloop_3m<C, V16>(sm, f, H, ldh, n, X, ldx, ncols, i0, j0, ka, kb);
  else if constexpr (C::KIND == 2)
    tile_mainloop_real<T, C, V16>(sm, f, H, ldh, n, X, ldx, ncols, i0, j0, ka, kb);
  else
    tile_mainloop_4m<T, C, V16>(sm, f, H, ldh, n, X, ldx, ncols, i0, j0, ka, kb);
}

template <typename T, class C, typename Fn>
__device__ __forceinline__ void tile_foreach(const typename C::Frag& f, Fn&& fn) {
  if constexpr (C::KIND == 1)
    tile_foreach_3m<C>(f, fn);
  else if constexpr (C::KIND == 2)
    tile_foreach_real<T, C>(f, fn);
  else
    tile_foreach_4m<T, C>(f, fn);
}

// Tile t -> (row tile, column tile) in the grouped order of grouped_tile (blocks of 8 row tiles,
// walked column tile by column tile).
__device__ __forceinline__ void tile_coords(int64_t t, int tiles_m, int tiles_n, int* tile_m,
                                            int* tile_n) {
  const TileMN c = grouped_tile(t, tiles_m, tiles_n);
  *tile_m = static_cast<int>(c.m);
  *tile_n = static_cast<int>(c.n);
}

// OUT <- alpha*HX + gamma*X + beta*OUT at (row, col); OUT is not read when beta == 0.
template <typename T>
__device__ __forceinline__ void epilogue_store(const T* __restrict__ X, int64_t ldx,
                                               T* __restrict__ OUT, int64_t ldo, int row, int col,
                                               T hre, T him, T alpha, T beta, T gamma) {
  using v2 = typename Acc<T>::v2;
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

// Real data: OUT <- alpha*HX + gamma*X + beta*OUT at (row, col).
template <typename T>
__device__ __forceinline__ void epilogue_store_real(const T* __restrict__ X, int64_t ldx,
                                                    T* __restrict__ OUT, int64_t ldo, int row,
                                                    int col, T v, T alpha, T beta, T gamma) {
  const T x = X[static_cast<int64_t>(row) + static_cast<int64_t>(col) * ldx];
  T* o = OUT + static_cast<int64_t>(row) + static_cast<int64_t>(col) * ldo;
  T r = alpha * v + gamma * x;
  if (beta != T(0)) r += beta * *o;
  *o = r;
}

// The epilogue of the tile's element type (complex interleaved or real).
template <typename T, class C>
__device__ __forceinline__ void store_result(const T* __restrict__ X, int64_t ldx,
                                             T* __restrict__ OUT, int64_t ldo, int row, int col,
                                             T hre, T him, T alpha, T beta, T gamma) {
  if constexpr (C::KIND == 2)
    epilogue_store_real<T>(X, ldx, OUT, ldo, row, col, hre, alpha, beta, gamma);
  else
    epilogue_store<T>(X, ldx, OUT, ldo, row, col, hre, him, alpha, beta, gamma);
}

// Values per output element: 2 for complex tiles, 1 for real ones.
template <class C> constexpr int elem_width() { return C::KIND == 2 ? 1 : 2; }

// Data-parallel schedule: one workgroup per output tile, in the XCD-aware order of dp_tile over
// the grouped tile order: the 16 workgroups an XCD starts together cover 8 row panels of H and
// 2 column panels of X, which they stream through that XCD's L2 at about the same time.
template <typename T, class C, int OCC, bool V16>
__global__ __launch_bounds__(kThreads, OCC) void hemm_dp_kernel(
    const T* __restrict__ H, int64_t ldh, int n, const T* __restrict__ X, int64_t ldx,
    T* __restrict__ OUT, int64_t ldo, int ncols, T alpha, T beta, T gamma, int tiles_m) {
  __shared__ typename C::Smem sm;
  typename C::Frag f;
  int tile_m, tile_n;
  tile_coords(dp_tile(blockIdx.x, gridDim.x), tiles_m, (ncols + C::BNC - 1) / C::BNC, &tile_m,
              &tile_n);
  const int i0 = tile_m * C::BMC, j0 = tile_n * C::BNC;
  const int nk = (n + C::KT - 1) / C::KT;
  tile_mainloop<T, C, V16>(sm, f, H, ldh, n, X, ldx, ncols, i0, j0, 0, nk);
  tile_foreach<T, C>(f, [&](int r, int c, T hre, T him) {
    if (i0 + r < n && j0 + c < ncols)
      store_result<T, C>(X, ldx, OUT, ldo, i0 + r, j0 + c, hre, him, alpha, beta, gamma);
  });
}

// Hybrid data-parallel + stream-K schedule on P persistent workgroups.
//   Phase 1: the first dp_tiles = floor(tiles / P) * P tiles, round-robin (workgroup p takes
//            tiles p, p + P, ...), each finished in place.
//   Phase 2: the remaining tiles' work units (tile, K stage), numbered u = (t - dp_tiles) * nk + kt,
//            split evenly: workgroup p owns [u0(p), u1(p)) with u0(p) = floor(p U / P).  A tile
//            covered by one workgroup is finished in place; otherwise each contributor writes its
//            partial sum H X (before the epilogue) to its own slot -- slot 0 for the segment in
//            the tile containing u0(p), slot 1 for the segment in the tile containing u1(p) - 1 --
//            and hemm_fixup_kernel adds the slots in increasing p, so the result does not depend
//            on timing.

// The integer schedule (sk_start, sk_owner, sk_segment, sk_slot, sk_fixup_tile, xcd_order) is
// shared with the host and checked on the CPU; it lives in host_logic.h.

template <typename T, class C, int OCC, bool V16>
__global__ __launch_bounds__(kThreads, OCC) void hemm_sk_kernel(
    const T* __restrict__ H, int64_t ldh, int n, const T* __restrict__ X, int64_t ldx,
    T* __restrict__ OUT, int64_t ldo, int ncols, T alpha, T beta, T gamma, int tiles_m,
    int nk, int64_t dp_tiles, int64_t units, T* __restrict__ partial) {
  __shared__ typename C::Smem sm;
  typename C::Frag f;
  const int64_t P = gridDim.x, p = blockIdx.x;
  const int tiles_n = (ncols + C::BNC - 1) / C::BNC;
  // Workgroups are dealt round-robin to the 8 XCDs (each with its own L2); q renumbers them so
  // that the workgroups of one XCD hold consecutive positions of the grouped tile order, i.e. a
  // block of few row panels of H and column panels of X, which they stream through that XCD's
  // L2 at the same time.
  const int64_t q = xcd_order(p, P);
  for (int64_t t = q; t < dp_tiles; t += P) {
    int tile_m, tile_n;
    tile_coords(t, tiles_m, tiles_n, &tile_m, &tile_n);
    const int i0 = tile_m * C::BMC, j0 = tile_n * C::BNC;
    tile_mainloop<T, C, V16>(sm, f, H, ldh, n, X, ldx, ncols, i0, j0, 0, nk);
    tile_foreach<T, C>(f, [&](int r, int c, T hre, T him) {
      if (i0 + r < n && j0 + c < ncols)
        store_result<T, C>(X, ldx, OUT, ldo, i0 + r, j0 + c, hre, him, alpha, beta, gamma);
    });
  }
  if (units == 0) return;
  const int64_t u0 = sk_start(p, units, P), u1 = sk_start(p + 1, units, P);
  constexpr int TE = C::BMC * C::BNC;  // output elements per tile
  int64_t u = u0;
  while (u < u1) {
    const SkSegment sg = sk_segment(u, u1, nk);
    const int64_t tr = sg.tile;  // tile index within the stream-K part
    const int ka = sg.ka, kb = sg.kb;
    const int64_t t = dp_tiles + tr;
    int tile_m, tile_n;
    tile_coords(t, tiles_m, tiles_n, &tile_m, &tile_n);
    const int i0 = tile_m * C::BMC, j0 = tile_n * C::BNC;
    tile_mainloop<T, C, V16>(sm, f, H, ldh, n, X, ldx, ncols, i0, j0, ka, kb);
    if (ka == 0 && kb == nk) {
      tile_foreach<T, C>(f, [&](int r, int c, T hre, T him) {
        if (i0 + r < n && j0 + c < ncols)
          store_result<T, C>(X, ldx, OUT, ldo, i0 + r, j0 + c, hre, him, alpha, beta, gamma);
      });
    } else {
      constexpr int EW = elem_width<C>();
      T* dst = partial + EW * (p * 2 + sk_slot(p, tr, units, P, nk)) * TE;
      tile_foreach<T, C>(f, [&](int r, int c, T hre, T him) {
        dst[EW * (r + c * C::BMC)] = hre;
        if constexpr (EW == 2) dst[EW * (r + c * C::BMC) + 1] = him;
      });
    }
    u = tr * nk + kb;
  }
}

// Element slices of a tile in the fixup: at most 4 elements per thread in each slice.
template <class C>
constexpr int fixup_slices() {
  constexpr int TE = C::BMC * C::BNC;
  return TE / (4 * kThreads) > 0 ? TE / (4 * kThreads) : 1;
}

// Grid = P x fixup_slices: workgroup (p, s) completes slice s of the split tile that contains
// u0(p), when p is the first workgroup whose range starts inside that tile.
template <typename T, class C>
__global__ __launch_bounds__(kThreads) void hemm_fixup_kernel(
    const T* __restrict__ X, int64_t ldx, T* __restrict__ OUT, int64_t ldo, int n, int ncols,
    T alpha, T beta, T gamma, int tiles_m, int nk, int64_t dp_tiles, int64_t units, int64_t P,
    const T* __restrict__ partial) {
  const int64_t tr = sk_fixup_tile(blockIdx.x, units, P, nk);
  if (tr < 0) return;
  const int64_t pf = sk_owner(tr * nk, units, P), pl = sk_owner((tr + 1) * nk - 1, units, P);
  const int64_t t = dp_tiles + tr;
  int tile_m, tile_n;
  tile_coords(t, tiles_m, (ncols + C::BNC - 1) / C::BNC, &tile_m, &tile_n);
  const int i0 = tile_m * C::BMC, j0 = tile_n * C::BNC;
  constexpr int TE = C::BMC * C::BNC;
  constexpr int SL = fixup_slices<C>();
  constexpr int ES = TE / SL;                          // elements per slice
  static_assert(ES * SL == TE && ES % kThreads == 0, "slice split");
  constexpr int EPT = ES / kThreads;                   // elements per thread
  constexpr int UNR = 4;                               // contributors whose loads are in flight
  constexpr int EW = elem_width<C>();
  const int e0 = static_cast<int>(blockIdx.y) * ES;
  // The slot offsets of up to kThreads contributors at a time (integer divisions) are found in
  // parallel, one per thread, into LDS.  The loads of UNR contributors are issued before any of
  // them is added; every element still adds its slots in increasing pp, and an empty range
  // (offset -1) adds nothing.
  __shared__ int64_t soff[kThreads];
  T hre[EPT], him[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) hre[q] = T(0), him[q] = T(0);
  for (int64_t c0 = pf; c0 <= pl; c0 += kThreads) {
    const int cnt = static_cast<int>(pl - c0 + 1 < kThreads ? pl - c0 + 1 : kThreads);
    __syncthreads();  // the previous chunk's offsets are consumed
    if (static_cast<int>(threadIdx.x) < cnt) {
      const int64_t pp = c0 + threadIdx.x;
      const int64_t a = sk_start(pp, units, P), b = sk_start(pp + 1, units, P);
      soff[threadIdx.x] = a >= b ? int64_t{-1} : EW * (pp * 2 + sk_slot(pp, tr, units, P, nk)) * TE;
    }
    __syncthreads();
    for (int j = 0; j < cnt; j += UNR) {
      T vre[UNR][EPT], vim[UNR][EPT];
      int64_t o[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        o[u] = j + u < cnt ? soff[j + u] : int64_t{-1};
        const T* src = partial + (o[u] < 0 ? 0 : o[u]);
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          const int e = e0 + static_cast<int>(threadIdx.x) + q * kThreads;
          vre[u][q] = o[u] < 0 ? T(0) : src[EW * e];
          if constexpr (EW == 2) vim[u][q] = o[u] < 0 ? T(0) : src[EW * e + 1];
        }
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u)
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          hre[q] = o[u] < 0 ? hre[q] : hre[q] + vre[u][q];
          if constexpr (EW == 2) him[q] = o[u] < 0 ? him[q] : him[q] + vim[u][q];
        }
    }
  }
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = e0 + static_cast<int>(threadIdx.x) + q * kThreads;
    const int r = e % C::BMC, c = e / C::BMC;
    if (i0 + r < n && j0 + c < ncols)
      store_result<T, C>(X, ldx, OUT, ldo, i0 + r, j0 + c, hre[q], him[q], alpha, beta, gamma);
  }
}

// Grouped schedule: one launch runs one product for each of up to kMaxGroup independent
// problems (continuous batching of small solves).  The tiles of all problems are concatenated.
// A product with ksplit > 1 has each output tile computed as ksplit K slices (workgroup
// tile + tiles * slice covers the K stages [slice * nk / ksplit, (slice + 1) * nk / ksplit)),
// whose partial sums go to the scratch; hemm_group_fixup_kernel adds them in slice order.  The
// split of a product depends only on its own n and ncols, so a problem's result does not
// depend on what it was grouped with.
template <typename T, class C, int OCC, bool V16>
__global__ __launch_bounds__(kThreads, OCC) void hemm_group_kernel(GroupArgs<T> args) {
  __shared__ typename C::Smem sm;
  typename C::Frag f;
  const int b = static_cast<int>(blockIdx.x);
  int g = 0;
  while (g + 1 < args.count && b >= args.d[g + 1].tile_begin) ++g;
  const GroupDesc<T> d = args.d[g];
  const int local = b - d.tile_begin;
  const int tiles_m = (d.n + C::BMC - 1) / C::BMC;
  const int tiles = tiles_m * ((d.ncols + C::BNC - 1) / C::BNC);
  const int S = d.ksplit > 1 ? d.ksplit : 1;
  const int tile = local % tiles, slice = local / tiles;
  const int tile_m = tile % tiles_m, tile_n = tile / tiles_m;
  const int i0 = tile_m * C::BMC, j0 = tile_n * C::BNC;
  const int nk = (d.n + C::KT - 1) / C::KT;
  const int ka = static_cast<int>(static_cast<int64_t>(slice) * nk / S);
  const int kb = static_cast<int>(static_cast<int64_t>(slice + 1) * nk / S);
  tile_mainloop<T, C, V16>(sm, f, d.H, d.ldh, d.n, d.X, d.ldx, d.ncols, i0, j0, ka, kb);
  if (S == 1) {
    tile_foreach<T, C>(f, [&](int r, int c, T hre, T him) {
      if (i0 + r < d.n && j0 + c < d.ncols)
        store_result<T, C>(d.X, d.ldx, d.OUT, d.ldo, i0 + r, j0 + c, hre, him, d.alpha, d.beta,
                          d.gamma);
    });
  } else {
    constexpr int EW = elem_width<C>();
    constexpr int TE = C::BMC * C::BNC;
    T* dst = args.partial + d.part_off + static_cast<int64_t>(slice * tiles + tile) * EW * TE;
    tile_foreach<T, C>(f, [&](int r, int c, T hre, T him) {
      dst[EW * (r + c * C::BMC)] = hre;
      if constexpr (EW == 2) dst[EW * (r + c * C::BMC) + 1] = him;
    });
  }
}

// Completes the K-sliced tiles of a grouped launch: workgroup fix_begin + fixup_slices * tile +
// e of a product adds the ksplit partial sums of element slice e of that tile, in slice order,
// and applies the epilogue.
template <typename T, class C>
__global__ __launch_bounds__(kThreads) void hemm_group_fixup_kernel(GroupArgs<T> args) {
  const int b = static_cast<int>(blockIdx.x);
  int g = -1;
  for (int q = 0; q < args.count; ++q)
    if (args.d[q].ksplit > 1 && b >= args.d[q].fix_begin) g = q;
  if (g < 0) return;
  const GroupDesc<T> d = args.d[g];
  constexpr int TE = C::BMC * C::BNC;
  constexpr int SL = fixup_slices<C>();
  constexpr int ES = TE / SL;
  static_assert(ES * SL == TE && ES % kThreads == 0, "slice split");
  constexpr int EPT = ES / kThreads;
  constexpr int EW = elem_width<C>();
  const int tiles_m = (d.n + C::BMC - 1) / C::BMC;
  const int tiles = tiles_m * ((d.ncols + C::BNC - 1) / C::BNC);
  const int local = b - d.fix_begin;
  const int tile = local / SL, es = local % SL;
  if (tile >= tiles) return;
  const int i0 = (tile % tiles_m) * C::BMC, j0 = (tile / tiles_m) * C::BNC;
  T hre[EPT], him[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) hre[q] = T(0), him[q] = T(0);
  for (int sl = 0; sl < d.ksplit; ++sl) {
    const T* src = args.partial + d.part_off + static_cast<int64_t>(sl * tiles + tile) * EW * TE;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = es * ES + static_cast<int>(threadIdx.x) + q * kThreads;
      hre[q] += src[EW * e];
      if constexpr (EW == 2) him[q] += src[EW * e + 1];
    }
  }
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = es * ES + static_cast<int>(threadIdx.x) + q * kThreads;
    const int r = e % C::BMC, c = e / C::BMC;
    if (i0 + r < d.n && j0 + c < d.ncols)
      store_result<T, C>(d.X, d.ldx, d.OUT, d.ldo, i0 + r, j0 + c, hre[q], him[q], d.alpha,
                        d.beta, d.gamma);
  }
}

template <typename T, class C, int OCC, bool V16 = false>
hipError_t launch_dp(const T* H, int64_t ldh, int64_t n, const T* X, int64_t ldx, T* OUT,
                     int64_t ldo, int64_t ncols, T alpha, T beta, T gamma, hipStream_t stream) {
  const int tiles_m = static_cast<int>((n + C::BMC - 1) / C::BMC);
  const int tiles_n = static_cast<int>((ncols + C::BNC - 1) / C::BNC);
  const int64_t blocks = static_cast<int64_t>(tiles_m) * tiles_n;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((hemm_dp_kernel<T, C, OCC, V16>), dim3(static_cast<unsigned>(blocks)),
                     dim3(kThreads), 0, stream, H, ldh, static_cast<int>(n), X, ldx, OUT, ldo,
                     static_cast<int>(ncols), alpha, beta, gamma, tiles_m);
  return hipGetLastError();
}

// Bytes of partial-sum scratch the stream-K schedule needs for P persistent workgroups.
template <typename T, class C>
constexpr size_t sk_scratch_bytes(int64_t P) {
  return static_cast<size_t>(P) * 2 * C::BMC * C::BNC * elem_width<C>() * sizeof(T);
}

template <typename T, class C, int OCC, bool V16 = false>
hipError_t launch_sk(const T* H, int64_t ldh, int64_t n, const T* X, int64_t ldx, T* OUT,
                     int64_t ldo, int64_t ncols, T alpha, T beta, T gamma, int64_t P, T* partial,
                     hipStream_t stream, bool hybrid = true) {
  const int tiles_m = static_cast<int>((n + C::BMC - 1) / C::BMC);
  const int tiles_n = static_cast<int>((ncols + C::BNC - 1) / C::BNC);
  const int nk = static_cast<int>((n + C::KT - 1) / C::KT);
  const int64_t tiles = static_cast<int64_t>(tiles_m) * tiles_n;
  const SkPlan plan = sk_plan(tiles, nk, P, hybrid);
  const int64_t dp_tiles = plan.dp_tiles, units = plan.units;
  P = plan.P;
  hipLaunchKernelGGL((hemm_sk_kernel<T, C, OCC, V16>), dim3(static_cast<unsigned>(P)), dim3(kThreads), 0,
                     stream, H, ldh, static_cast<int>(n), X, ldx, OUT, ldo,
                     static_cast<int>(ncols), alpha, beta, gamma, tiles_m, nk, dp_tiles, units,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || units == 0) return e;
  hipLaunchKernelGGL((hemm_fixup_kernel<T, C>),
                     dim3(static_cast<unsigned>(P), static_cast<unsigned>(fixup_slices<C>())),
                     dim3(kThreads), 0, stream, X, ldx, OUT, ldo, static_cast<int>(n), static_cast<int>(ncols), alpha,
                     beta, gamma, tiles_m, nk, dp_tiles, units, P, partial);
  return hipGetLastError();
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


namespace {
// Tile shapes (complex rows x complex columns, K stage, wave grid).  Both precisions use the
// same wide tile; columns <= 32 use the narrow one.
// LDS rows are padded by 2 doubles (FP64) or 8 floats (FP32: keeps 16-byte aligned rows for
// the two-element vector loads).
// The FP64 wide tile interleaves the next stage's LDS stores with its last K step's MFMAs.
template <typename T>
using WideTile = Tile<T, 64, 64, 16, 2, 2, sizeof(T) == 4 ? 8 : 2, 0, false, -1, sizeof(T) == 4 ? 0 : 1>;
template <typename T> using NarrowTile = Tile<T, 64, 32, 16, 4, 1, sizeof(T) == 4 ? 8 : 2>;
// FP64 thin tile for <= 16 columns (the Lanczos block, a filter's last columns): 128 complex
// rows x 16 columns, so a thin product pads half as many columns as the narrow tile and its
// MFMA work drops below the time to stream H.
using ThinTile64 = Tile<double, 128, 16, 16, 4, 1, 2>;
// FP64 slim tile: 32 columns, K stages of 8, four workgroups per CU (125 VGPRs, 25 KB LDS); the
// next stage's global loads and LDS stores are both interleaved with MFMAs.  Padding the
// columns to 32 instead of 64 wastes less work on ragged widths, but it moves more operand data
// per flop: with full-precision operands (where the chip runs at its power limit) it is about
// 7 % slower per executed flop than the wide tile.  It is chosen only when padding to 64 would
// waste over 10 % more work than padding to 32.
using SlimTile64 = Tile<double, 64, 32, 8, 2, 2, 2, 0, false, 1, 2>;
constexpr int kOccSlim = 4;
// Real tiles: 128 x 128 real outputs (the complex wide tile's register and LDS footprint); a
// 256 x 16 tile for the thin blocks of the Lanczos runs.
template <typename T> using RealTile = TileR<T, 128, 128, 16, 2, 2, sizeof(T) == 4 ? 4 : 2>;
template <typename T> using RealThinTile = TileR<T, 256, 16, 16, 4, 1, sizeof(T) == 4 ? 4 : 2>;
constexpr double kSlimCost = 1.10;

// 3M tile for the planar FP32 products: FP64 promotion every eight stages (128 K terms), three
// workgroups per CU (the combined promotion keeps it at 163 VGPRs).  Each promotion waits for
// the MFMA pipeline to drain: promoting every 4 stages instead of 2 ran about 9 % faster, every
// 8 instead of 4 another 2-3 % (orders 10000-20000).  The FP32 part of the error grows like
// sqrt(128) units of FP32 roundoff within a chunk, far below the rounding of the inputs to FP32
// and the 1e-6 residual at which the mixed solver leaves FP32.
using Wide3M = Tile3M<64, 64, 16, 2, 2, 4, 8, float, 3>;
// The same 3M scheme on FP64 MFMA for complex128 data stored as two float64 planes: three
// real products instead of four per complex product.  No promotion (FP64 accumulators);
// 8-byte loads (measured faster than 16-byte ones for this tile); K stages of 8 with three
// workgroups per CU (35 KB of LDS, at most 168 VGPRs), 4-6 % faster than stages of 16 with two.
using Wide3M64 = Tile3M<64, 64, 8, 2, 2, 4, 0, double, 3>;
using Narrow3M64 = Tile3M<64, 32, 16, 4, 1, 4, 0, double>;
using Thin3M64 = Tile3M<128, 16, 16, 4, 1, 4, 0, double>;

// Two-element (16-byte) global loads are used for complex64 data when H and X are 16-byte
// aligned and n and their leading dimensions are even.
template <typename T>
bool use_v16(const T* H, int64_t ldh, const T* X, int64_t ldx, int64_t n) {
  return sizeof(T) == 4 && (reinterpret_cast<uintptr_t>(H) % 16) == 0 &&
         (reinterpret_cast<uintptr_t>(X) % 16) == 0 && ldh % 2 == 0 && ldx % 2 == 0 && n % 2 == 0;
}
constexpr int kOcc = 2;  // workgroups per CU the tiles are built for

// Wide global loads: two-element units for complex64 (16 bytes) or for real data.
template <typename T, class C>
bool wide_loads(const T* H, int64_t ldh, const T* X, int64_t ldx, int64_t n) {
  if constexpr (C::KIND == 2)
    return (reinterpret_cast<uintptr_t>(H) % (2 * sizeof(T))) == 0 &&
           (reinterpret_cast<uintptr_t>(X) % (2 * sizeof(T))) == 0 && ldh % 2 == 0 &&
           ldx % 2 == 0 && n % 2 == 0;
  else
    return use_v16(H, ldh, X, ldx, n);
}

template <typename T, class C, int OCC = C::OCC>
hipError_t launch_sched(const T* H, int64_t ldh, int64_t n, const T* X, int64_t ldx, T* OUT,
                        int64_t ldo, int64_t ncols, T alpha, T beta, T gamma,
                        const ProductScratch& ps, hipStream_t stream, bool v16_ok = true) {
  const int64_t tiles = ((n + C::BMC - 1) / C::BMC) * ((ncols + C::BNC - 1) / C::BNC);
  const int64_t slots = static_cast<int64_t>(ps.cus) * OCC;
  const int64_t rounds = (tiles + slots - 1) / slots;
  const double eff = static_cast<double>(tiles) / static_cast<double>(rounds * slots);
  if (ps.sk_need) {
    if (eff < 0.92) *ps.sk_need = std::max(*ps.sk_need, sk_scratch_bytes<T, C>(slots));
    return hipSuccess;
  }
  const bool v16 = v16_ok && wide_loads<T, C>(H, ldh, X, ldx, n);
  if (eff >= 0.92 || !ps.ptr || sk_scratch_bytes<T, C>(slots) > ps.bytes) {
    if (v16)
      return launch_dp<T, C, OCC, true>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma,
                                        stream);
    return launch_dp<T, C, OCC>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, stream);
  }
  if (v16)
    return launch_sk<T, C, OCC, true>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma,
                                      slots, static_cast<T*>(ps.ptr), stream);
  return launch_sk<T, C, OCC>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, slots,
                              static_cast<T*>(ps.ptr), stream);
}
}  // namespace

// Stream-K partial sums of a tile on a device with `cus` compute units.
template <typename T, class C>
size_t tile_scratch(int cus, int occ = C::OCC) {
  return sk_scratch_bytes<T, C>(static_cast<int64_t>(cus) * occ);
}

size_t product_scratch_bytes(int cus) {
  size_t b = tile_scratch<double, WideTile<double>>(cus);
  b = std::max(b, tile_scratch<float, WideTile<float>>(cus));
  b = std::max(b, tile_scratch<double, NarrowTile<double>>(cus));
  b = std::max(b, tile_scratch<double, SlimTile64>(cus, kOccSlim));
  b = std::max(b, tile_scratch<double, ThinTile64>(cus));
  b = std::max(b, tile_scratch<float, Wide3M>(cus));
  b = std::max(b, tile_scratch<double, Wide3M64>(cus));
  b = std::max(b, tile_scratch<double, Narrow3M64>(cus));
  b = std::max(b, tile_scratch<double, Thin3M64>(cus));
  b = std::max(b, tile_scratch<double, RealTile<double>>(cus));
  b = std::max(b, tile_scratch<double, RealThinTile<double>>(cus));
  return b;
}

template <typename T>
hipError_t launch_hemm_step_real(const T* H, int64_t ldh, int64_t n, const T* X, int64_t ldx,
                                 T* OUT, int64_t ldo, int64_t ncols, T alpha, T beta, T gamma,
                                 const ProductScratch& ps, hipStream_t stream) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  if (ncols <= 16)
    return launch_sched<T, RealThinTile<T>>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta,
                                            gamma, ps, stream);
  return launch_sched<T, RealTile<T>>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, ps,
                                      stream);
}
template hipError_t launch_hemm_step_real<double>(const double*, int64_t, int64_t, const double*,
                                                  int64_t, double*, int64_t, int64_t, double,
                                                  double, double, const ProductScratch&,
                                                  hipStream_t);
template hipError_t launch_hemm_step_real<float>(const float*, int64_t, int64_t, const float*,
                                                 int64_t, float*, int64_t, int64_t, float, float,
                                                 float, const ProductScratch&, hipStream_t);

template <typename T>
hipError_t launch_hemm_step(const T* H, int64_t ldh, int64_t n, const T* X, int64_t ldx, T* OUT,
                            int64_t ldo, int64_t ncols, T alpha, T beta, T gamma,
                            const ProductScratch& ps, hipStream_t stream) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 8) {
    // Columns padded to whole tiles: 32-wide slim tiles when that saves more than their lower
    // per-flop rate costs.
    if (ncols <= 16)
      return launch_sched<T, ThinTile64>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma,
                                         ps, stream);
    if (ncols <= 32)
      return launch_sched<T, NarrowTile<T>>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta,
                                            gamma, ps, stream);
    const double w64 = static_cast<double>((ncols + 63) / 64 * 64);
    const double w32 = static_cast<double>((ncols + 31) / 32 * 32);
    if (w32 * kSlimCost < w64)
      return launch_sched<T, SlimTile64, kOccSlim>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha,
                                                   beta, gamma, ps, stream);
    return launch_sched<T, WideTile<T>>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma,
                                        ps, stream);
  }
  if (ncols <= 32)
    return launch_sched<T, NarrowTile<T>>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma,
                                          ps, stream);
  return launch_sched<T, WideTile<T>>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, ps,
                                      stream);
}

// Grouped launches.  Workgroup slots of the whole device that a lone product's K split aims
// to fill, and the most K slices per tile (each slice keeps at least 8 K stages).
constexpr int kGroupSlots = 512;
constexpr int kGroupMaxSplit = 8;

// K slices of a product in a grouped launch: a function of n and ncols only.
template <class C>
int group_ksplit(int64_t n, int64_t ncols) {
  const int64_t tiles = ((n + C::BMC - 1) / C::BMC) * ((ncols + C::BNC - 1) / C::BNC);
  const int64_t nk = (n + C::KT - 1) / C::KT;
  int64_t s = tiles > 0 ? kGroupSlots / tiles : 1;
  s = std::min<int64_t>(s, kGroupMaxSplit);
  s = std::min<int64_t>(s, nk / 8);
  return static_cast<int>(std::max<int64_t>(s, 1));
}

// Partial-sum values of one product (all its slices).
template <typename T, class C>
int64_t group_partial_values(int64_t n, int64_t ncols) {
  const int s = group_ksplit<C>(n, ncols);
  if (s <= 1) return 0;
  const int64_t tiles = ((n + C::BMC - 1) / C::BMC) * ((ncols + C::BNC - 1) / C::BNC);
  return s * tiles * C::BMC * C::BNC * elem_width<C>();
}

// Runs the products in launches of at most kMaxGroup products whose partial sums fit the
// scratch; each launch is the main kernel and, when a product is split, the fixup kernel.
template <typename T, class C, bool V16>
hipError_t launch_group(const GroupDesc<T>* descs, int count, const GroupScratch& gs,
                        hipStream_t stream) {
  // Products that fill the device by themselves run alone on the single-product schedule; the
  // choice depends only on their own shape, so a product is computed the same way whatever else
  // is in the tick.
  auto alone = [&](const GroupDesc<T>& d) {
    const int64_t t = ((d.n + C::BMC - 1) / C::BMC) *
                      static_cast<int64_t>((d.ncols + C::BNC - 1) / C::BNC);
    return gs.cus > 0 && gs.ptr && 2 * t > kGroupSlots;
  };
  for (int q = 0; q < count; ++q) {
    const GroupDesc<T>& d = descs[q];
    if (d.n <= 0 || d.ncols <= 0 || !alone(d)) continue;
    ProductScratch ps;
    ps.ptr = gs.ptr;
    ps.bytes = gs.bytes;
    ps.cus = gs.cus;
    const hipError_t e = launch_sched<T, C>(d.H, d.ldh, d.n, d.X, d.ldx, d.OUT, d.ldo, d.ncols,
                                            d.alpha, d.beta, d.gamma, ps, stream, V16);
    if (e != hipSuccess) return e;
  }
  const int64_t cap = static_cast<int64_t>(gs.bytes / sizeof(T));
  int q0 = 0;
  while (q0 < count) {
    GroupArgs<T> a{};
    a.partial = static_cast<T*>(gs.ptr);
    int64_t tiles = 0, fix = 0, part = 0;
    int q = q0;
    for (; q < count && a.count < kMaxGroup; ++q) {
      const GroupDesc<T>& src = descs[q];
      if (src.n > 0 && src.ncols > 0 && alone(src)) continue;   // launched above
      const int64_t pv = group_partial_values<T, C>(src.n, src.ncols);
      if (pv > 0 && (!gs.ptr || pv > cap)) return hipErrorInvalidValue;   // scratch too small
      if (part + pv > cap) break;                                        // next launch
      GroupDesc<T> d = src;
      const int64_t t = ((d.n + C::BMC - 1) / C::BMC) *
                        static_cast<int64_t>((d.ncols + C::BNC - 1) / C::BNC);
      d.ksplit = group_ksplit<C>(d.n, d.ncols);
      d.tile_begin = static_cast<int>(tiles);
      d.fix_begin = static_cast<int>(fix);
      d.part_off = part;
      tiles += t * d.ksplit;
      if (d.ksplit > 1) fix += t * fixup_slices<C>();
      part += pv;
      a.d[a.count++] = d;
    }
    q0 = q;
    if (tiles == 0) continue;
    if (tiles > 0x7fffffff || fix > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((hemm_group_kernel<T, C, C::OCC, V16>), dim3(static_cast<unsigned>(tiles)),
                       dim3(kThreads), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (fix > 0) {
      hipLaunchKernelGGL((hemm_group_fixup_kernel<T, C>), dim3(static_cast<unsigned>(fix)),
                         dim3(kThreads), 0, stream, a);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_hemm_group(const GroupDesc<T>* descs, int count, const GroupScratch& gs,
                             hipStream_t stream) {
  bool v16 = true;
  for (int q = 0; q < count; ++q)
    v16 = v16 && use_v16(descs[q].H, descs[q].ldh, descs[q].X, descs[q].ldx, descs[q].n);
  if (v16) return launch_group<T, WideTile<T>, true>(descs, count, gs, stream);
  return launch_group<T, WideTile<T>, false>(descs, count, gs, stream);
}
template hipError_t launch_hemm_group<double>(const GroupDesc<double>*, int, const GroupScratch&,
                                              hipStream_t);
template hipError_t launch_hemm_group<float>(const GroupDesc<float>*, int, const GroupScratch&,
                                             hipStream_t);

hipError_t launch_hemm_step_3m(const float* H, int64_t ldh, int64_t n, const float* X,
                               int64_t ldx, float* OUT, int64_t ldo, int64_t ncols, float alpha,
                               float beta, float gamma, const ProductScratch& ps,
                               hipStream_t stream) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  // vector loads of four rows per plane need ldh % 4 == 0 on top of the usual conditions
  return launch_sched<float, Wide3M>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma, ps,
                                     stream, ldh % 4 == 0);
}

hipError_t launch_hemm_step_3m_f64(const double* H, int64_t ldh, int64_t n, const double* X,
                                   int64_t ldx, double* OUT, int64_t ldo, int64_t ncols,
                                   double alpha, double beta, double gamma,
                                   const ProductScratch& ps, hipStream_t stream) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  if (ncols <= 16)
    return launch_sched<double, Thin3M64>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma,
                                          ps, stream, false);
  if (ncols <= 32)
    return launch_sched<double, Narrow3M64>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta,
                                            gamma, ps, stream, false);
  return launch_sched<double, Wide3M64>(H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma,
                                        ps, stream, false);
}

hipError_t launch_hemm_group_3m(const GroupDesc<float>* descs, int count, const GroupScratch& gs,
                                hipStream_t stream) {
  // vector loads of four rows per plane need ldh % 4 == 0 on top of the usual conditions
  bool v16 = true;
  for (int q = 0; q < count; ++q)
    v16 = v16 && descs[q].ldh % 4 == 0 &&
          use_v16(descs[q].H, descs[q].ldh, descs[q].X, descs[q].ldx, descs[q].n);
  if (v16) return launch_group<float, Wide3M, true>(descs, count, gs, stream);
  return launch_group<float, Wide3M, false>(descs, count, gs, stream);
}

hipError_t launch_hemm_group_3m_f64(const GroupDesc<double>* descs, int count,
                                    const GroupScratch& gs, hipStream_t stream) {
  return launch_group<double, Wide3M64, false>(descs, count, gs, stream);
}

size_t group_scratch_min_bytes() {
  // a split product has fewer than kGroupSlots tiles and at most kGroupSlots / tiles slices, so
  // its partial sums hold at most kGroupSlots tiles' worth of values
  size_t b = 0;
  b = std::max(b, kGroupSlots * sizeof(double) * 2 * WideTile<double>::BMC * WideTile<double>::BNC);
  b = std::max(b, kGroupSlots * sizeof(float) * 2 * WideTile<float>::BMC * WideTile<float>::BNC);
  b = std::max(b, kGroupSlots * sizeof(float) * 2 * Wide3M::BMC * Wide3M::BNC);
  b = std::max(b, kGroupSlots * sizeof(double) * 2 * Wide3M64::BMC * Wide3M64::BNC);
  return b;
}

template hipError_t launch_hemm_step<double>(const double*, int64_t, int64_t, const double*,
                                             int64_t, double*, int64_t, int64_t, double, double,
                                             double, const ProductScratch&, hipStream_t);
template hipError_t launch_hemm_step<float>(const float*, int64_t, int64_t, const float*, int64_t,
                                            float*, int64_t, int64_t, float, float, float,
                                            const ProductScratch&, hipStream_t);

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

namespace {
template <typename S, typename D>
__global__ void convert_real_kernel(const S* __restrict__ src, int64_t lds, D* __restrict__ dst,
                                    int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = t % rows, c = t / rows;
    dst[r + c * ldd] = static_cast<D>(src[r + c * lds]);
  }
}
}  // namespace

hipError_t launch_convert_f64_to_f32(const double* src, int64_t lds, float* dst, int64_t ldd,
                                     int64_t rows, int64_t cols, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL((convert_real_kernel<double, float>), dim3(convert_blocks(rows * cols)),
                     dim3(256), 0, stream, src, lds, dst, ldd, rows, cols);
  return hipGetLastError();
}

hipError_t launch_convert_f32_to_f64(const float* src, int64_t lds, double* dst, int64_t ldd,
                                     int64_t rows, int64_t cols, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL((convert_real_kernel<float, double>), dim3(convert_blocks(rows * cols)),
                     dim3(256), 0, stream, src, lds, dst, ldd, rows, cols);
  return hipGetLastError();
}

namespace {
__global__ void planar_kernel(const double* __restrict__ src, int64_t lds, float* __restrict__ dst,
                              int64_t ldd, int64_t n) {
  const int64_t total = n * n;
  float* im = dst + ldd * n;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = t % n, c = t / n;
    const double* s = src + 2 * (r + c * lds);
    dst[r + c * ldd] = static_cast<float>(s[0]);
    im[r + c * ldd] = static_cast<float>(s[1]);
  }
}
}  // namespace

namespace {
__global__ void planar64_kernel(const double* __restrict__ src, int64_t lds,
                                double* __restrict__ dst, int64_t ldd, int64_t n) {
  const int64_t total = n * n;
  double* im = dst + ldd * n;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = t % n, c = t / n;
    const double2 v = *reinterpret_cast<const double2*>(src + 2 * (r + c * lds));
    dst[r + c * ldd] = v.x;
    im[r + c * ldd] = v.y;
  }
}
}  // namespace

hipError_t launch_convert_c128_to_planar64(const double* src, int64_t lds, double* dst,
                                           int64_t ldd, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(planar64_kernel, dim3(convert_blocks(n * n)), dim3(256), 0, stream, src,
                     lds, dst, ldd, n);
  return hipGetLastError();
}

hipError_t launch_convert_c128_to_planar32(const double* src, int64_t lds, float* dst, int64_t ldd,
                                           int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(planar_kernel, dim3(convert_blocks(n * n)), dim3(256), 0, stream, src, lds,
                     dst, ldd, n);
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
