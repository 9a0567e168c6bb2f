// Host-side logic of the solver that needs no device: the filter's product schedule
// (Algorithm 4 / Eq. (7) scalars), Algorithm 5 (degrees), the small symmetric eigensolver for
// the Lanczos tridiagonals and the DoS estimate of Sec. 4.2 (Algorithm 6).  Header-only and free
// of HIP so that it can also be compiled and checked on a machine without a GPU.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

namespace chase {

// ---------------------------------------------------------------------------------------------
// Integer schedule of the product kernel's stream-K part (constexpr, so the kernels use these
// same functions).  U work units (tile, K stage), numbered tile-major, are split over P
// persistent workgroups: workgroup p owns [sk_start(p), sk_start(p + 1)).
constexpr int64_t sk_start(int64_t p, int64_t units, int64_t P) { return p * units / P; }
// The workgroup whose range contains unit u (the largest p with sk_start(p) <= u).
constexpr int64_t sk_owner(int64_t u, int64_t units, int64_t P) {
  return ((u + 1) * P - 1) / units;
}
// One segment of a workgroup's range: the units of one tile, K stages [ka, kb).
struct SkSegment {
  int64_t tile;
  int ka, kb;
};
constexpr SkSegment sk_segment(int64_t u, int64_t u1, int nk) {
  const int64_t tr = u / nk;
  const int ka = static_cast<int>(u - tr * nk);
  const int64_t rest = static_cast<int64_t>(ka) + (u1 - u);
  return {tr, ka, static_cast<int>(rest < nk ? rest : nk)};
}
// Partial-sum slot of workgroup p's segment in split tile tr: 0 for the tile holding its first
// unit, 1 for the tile holding its last.
constexpr int sk_slot(int64_t p, int64_t tr, int64_t units, int64_t P, int nk) {
  return sk_start(p, units, P) / nk == tr ? 0 : 1;
}
// The split tile that fixup workgroup q completes, or -1: q completes the tile containing its
// first unit when that unit is not the tile's first and no earlier workgroup's range starts
// inside the same tile.
constexpr int64_t sk_fixup_tile(int64_t q, int64_t units, int64_t P, int nk) {
  if (q == 0 || units == 0) return -1;
  const int64_t uq = sk_start(q, units, P);
  if (uq >= units || uq % nk == 0) return -1;
  const int64_t tr = uq / nk;
  if (sk_start(q - 1, units, P) > tr * nk) return -1;
  return tr;
}
// Hybrid plan for `tiles` output tiles of nk K stages on P persistent workgroups: the first
// dp_tiles = whole rounds of tiles go data-parallel, the rest is split as stream-K units; with
// no data-parallel round, P shrinks to the unit count so that no workgroup is idle.
struct SkPlan {
  int64_t dp_tiles, units, P;
};
constexpr SkPlan sk_plan(int64_t tiles, int nk, int64_t P, bool hybrid) {
  const int64_t dp = hybrid ? (tiles / P) * P : 0;
  const int64_t units = (tiles - dp) * nk;
  return {dp, units, (dp == 0 && P > units) ? units : P};
}
// Workgroup p's position in the data-parallel tile order: the workgroups dealt to one of the 8
// XCDs (round-robin by index) get consecutive positions.
constexpr int64_t xcd_order(int64_t p, int64_t P) {
  return (P % 8 == 0) ? (p % 8) * (P / 8) + p / 8 : p;
}

// Tile of workgroup b in a data-parallel grid of G workgroups.  Workgroups are dealt to the 8
// XCDs round-robin by index; in every full window of 8 * kDpChunk workgroups the ones dealt to
// one XCD get kDpChunk consecutive tiles (with column tiles varying fastest, the column tiles of
// the same row panels of H, which then share that XCD's L2).  The last partial window keeps
// the identity.  A bijection of [0, G).
constexpr int64_t kDpChunk = 16;
constexpr int64_t dp_tile(int64_t b, int64_t G) {
  const int64_t W = 8 * kDpChunk;
  const int64_t w = b / W;
  if ((w + 1) * W > G) return b;
  const int64_t r = b % W;
  return w * W + (r % 8) * kDpChunk + r / 8;
}

// Output tile at position t of the product kernels' tile order: groups of kTileGroupRows row
// tiles (the last group may be shorter), each walked column tile by column tile, row tiles
// fastest.  The workgroups one XCD runs together take consecutive positions (xcd_order,
// dp_tile), so they cover a block of few row panels of H and few column panels of X (16
// positions: 8 x 2 tiles, 96: 8 x 12) instead of all column tiles of one or two row panels,
// and fetch fewer distinct panels into that XCD's L2.  A bijection of [0, tiles_m tiles_n).
constexpr int64_t kTileGroupRows = 8;
struct TileMN {
  int64_t m, n;
};
constexpr TileMN grouped_tile(int64_t t, int64_t tiles_m, int64_t tiles_n) {
  const int64_t per_group = kTileGroupRows * tiles_n;
  const int64_t g = t / per_group;
  const int64_t first = g * kTileGroupRows;
  const int64_t rows = tiles_m - first < kTileGroupRows ? tiles_m - first : kTileGroupRows;
  const int64_t r = t - g * per_group;
  return {first + r % rows, r / rows};
}

// K-slices of a Gram product A^H B (m1 x m2 result, k rows) computed as a batch of slice
// products plus a sum: enough slices that about 512 output tiles of 64 x 64 are in flight
// (tall-skinny shapes leave most of the GPU idle otherwise), at most 16, each at least 256 rows.
constexpr int64_t gram_slices(int64_t m1, int64_t m2, int64_t k) {
  const int64_t tiles = ((m1 + 63) / 64) * ((m2 + 63) / 64);
  int64_t p = tiles > 0 ? (512 + tiles - 1) / tiles : 1;
  if (p > 16) p = 16;
  if (p > k / 256) p = k / 256;
  return p < 1 ? 1 : p;
}
// Elements of the slice buffer reserved for Gram products of at most nb x nb; a product whose
// slices would not fit uses fewer slices (never fewer than 1: the buffer holds nb * nb).
constexpr int64_t gram_buffer_elems(int64_t nb) {
  const int64_t a = 16 * nb * nb, b = (int64_t{1} << 21) + nb * nb;
  return a < b ? a : b;
}

// One product of Algorithm 4: OUT[:, col0:col0+ncols] <- alpha H X + gamma X + beta OUT where
// (X, OUT) = (V, W) when from_v, else (W, V).
struct FilterProduct {
  bool from_v;
  int64_t col0, ncols;
  double alpha, beta, gamma;
};

// The products of one filter call on sorted even degrees (the recurrence scalars of Eq. (7)),
// handed one by one to fn(const FilterProduct&) without building a list (no allocation).
template <class Fn>
inline void for_each_filter_product(int64_t ncols, const int32_t* degrees, double b_sup,
                                    double mu_1, double mu_nevnex, Fn&& fn) {
  if (ncols <= 0) return;
  const double c = 0.5 * (b_sup + mu_nevnex);
  const double e = 0.5 * (b_sup - mu_nevnex);
  const double sigma1 = e / (mu_1 - c);
  const int32_t m_max = degrees[ncols - 1];
  // product 1, every column: W <- a1 H V + g1 V
  double alpha = sigma1 / e;
  fn(FilterProduct{/*from_v=*/true, 0, ncols, alpha, 0.0, -alpha * c});
  bool in_is_w = true;  // p_{i-1} lives in W, p_{i-2} in V
  double sigma = sigma1;
  int64_t s = 0;
  while (s < ncols && degrees[s] <= 1) ++s;
  for (int32_t i = 2; i <= m_max; ++i) {
    const double tau = 1.0 / (2.0 / sigma1 - sigma);
    alpha = 2.0 * tau / e;
    fn(FilterProduct{/*from_v=*/!in_is_w, s, ncols - s, alpha, -tau * sigma, -alpha * c});
    in_is_w = !in_is_w;
    sigma = tau;
    while (s < ncols && degrees[s] <= i) ++s;
  }
  // m_max is even, so the last product wrote V.
}

// The same products as a list.
inline std::vector<FilterProduct> filter_schedule(int64_t ncols, const int32_t* degrees, double b_sup,
                                                  double mu_1, double mu_nevnex) {
  std::vector<FilterProduct> out;
  for_each_filter_product(ncols, degrees, b_sup, mu_1, mu_nevnex,
                          [&](const FilterProduct& p) { out.push_back(p); });
  return out;
}


// Symmetric eigen-decomposition of a small dense matrix by cyclic Jacobi rotations (used for the
// k x k Lanczos tridiagonals; k is a few dozen).  a: row-major k x k, destroyed.  On return
// evals ascending and evecs[:, i] (row-major, column i) the matching eigenvectors.
inline void jacobi_eigh(int k, std::vector<double>& a, std::vector<double>& evals,
                 std::vector<double>& evecs) {
  std::vector<double> v(static_cast<size_t>(k) * k, 0.0);
  for (int i = 0; i < k; ++i) v[i * k + i] = 1.0;
  double fro = 0.0;
  for (double x : a) fro += x * x;
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) off += a[p * k + q] * a[p * k + q];
    if (std::sqrt(off) <= 1e-17 * fro) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = a[p * k + q];
        if (apq == 0.0) continue;
        const double theta = (a[q * k + q] - a[p * k + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < k; ++r) {  // columns p, q
          const double arp = a[r * k + p], arq = a[r * k + q];
          a[r * k + p] = c * arp - s * arq;
          a[r * k + q] = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {  // rows p, q
          const double apr = a[p * k + r], aqr = a[q * k + r];
          a[p * k + r] = c * apr - s * aqr;
          a[q * k + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double vrp = v[r * k + p], vrq = v[r * k + q];
          v[r * k + p] = c * vrp - s * vrq;
          v[r * k + q] = s * vrp + c * vrq;
        }
      }
  }
  std::vector<int> idx(k);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return a[x * k + x] < a[y * k + y]; });
  evals.resize(k);
  evecs.assign(static_cast<size_t>(k) * k, 0.0);
  for (int i = 0; i < k; ++i) {
    evals[i] = a[idx[i] * k + idx[i]];
    for (int r = 0; r < k; ++r) evecs[r * k + i] = v[r * k + idx[i]];
  }
}

struct LanczosRun {
  std::vector<double> ritz, evecs;  // evecs row-major k x k, column i = eigenvector i
  int k = 0;
  double beta_last = 0.0;
};

inline LanczosRun tridiag_eig(const std::vector<double>& al, const std::vector<double>& be, int nv, int c,
                       int k) {
  // truncate at the first vanishing beta (invariant subspace)
  int kk = k;
  for (int j = 0; j < k; ++j)
    if (!(be[j * nv + c] > 0.0)) {
      kk = j + 1;
      break;
    }
  std::vector<double> T(static_cast<size_t>(kk) * kk, 0.0);
  for (int j = 0; j < kk; ++j) {
    T[j * kk + j] = al[j * nv + c];
    if (j + 1 < kk) T[j * kk + j + 1] = T[(j + 1) * kk + j] = be[j * nv + c];
  }
  LanczosRun r;
  r.k = kk;
  r.beta_last = be[(kk - 1) * nv + c];
  jacobi_eigh(kk, T, r.ritz, r.evecs);
  return r;
}

// mu_{nev+nex} from the Gaussian-smoothed spectral density of the DoS runs (Sec. 4.2, Eq. (10)):
// bisection on sum_i w_i Phi((t - lambda_i)/s) = (nev+nex)/n.
inline double dos_mu(const std::vector<LanczosRun>& runs, double lo, double b_sup, double sigma,
              double target) {
  const double half = b_sup > lo ? 0.5 * (b_sup - lo) : 1.0;
  const double s = sigma * half;
  auto cdf = [&](double t) {
    double acc = 0.0;
    for (const auto& r : runs)
      for (int i = 0; i < r.k; ++i) {
        const double w = r.evecs[0 * r.k + i] * r.evecs[0 * r.k + i];
        acc += w * 0.5 * (1.0 + std::erf((t - r.ritz[i]) / (s * std::sqrt(2.0))));
      }
    return acc / static_cast<double>(runs.size());
  };
  double a = lo - 8.0 * s, b = b_sup + 8.0 * s;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (a + b);
    if (cdf(mid) < target)
      a = mid;
    else
      b = mid;
  }
  return 0.5 * (a + b);
}

// Algorithm 5 for one vector.
inline int degree_of(double tol, double res, double ritz, double c, double e, int deg_extra, int deg_max) {
  const double t = (ritz - c) / e;
  double rho;
  if (std::fabs(t) <= 1.0) {
    rho = 1.0;
  } else {
    const double r = std::sqrt(t * t - 1.0);
    rho = std::max(std::fabs(t - r), std::fabs(t + r));
  }
  const double lr = std::log(rho);
  int d;
  if (!(lr > 0.0) || !(res > 0.0)) {
    d = deg_max;
  } else {
    const double q = std::fabs(std::log(res / tol) / lr);
    const double dd = std::ceil(q) + deg_extra;
    d = dd > deg_max ? deg_max : static_cast<int>(dd);
  }
  return d + (d & 1);
}


}  // namespace chase
