// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/chase.h"
#include "host_logic.h"

namespace chase {

// Partial-sum scratch of the stream-K product schedule (owned by the context, fixed size).
struct ProductScratch {
  void* ptr = nullptr;
  size_t bytes = 0;
  int cus = 0;  // compute units of the device
  // Dry run: when set, the product launchers enqueue nothing and raise *sk_need to the
  // partial-sum bytes the stream-K schedule they would choose needs (0 for a data-parallel
  // grid), so a caller with a fixed scratch can check a whole filter call before launching it.
  size_t* sk_need = nullptr;
};
size_t product_scratch_bytes(int cus);

// ----------------------------------------------------------------------------- kernels
// One fused complex product  OUT <- alpha*H*X + gamma*X + beta*OUT  on ncols columns.
// T = double (complex128 data) or float (complex64 data); pointers address interleaved
// (re, im) pairs, leading dimensions count complex elements.
template <typename T>
hipError_t launch_hemm_step(const T* H, int64_t ldh, int64_t n, const T* X, int64_t ldx, T* OUT,
                            int64_t ldo, int64_t ncols, T alpha, T beta, T gamma,
                            const ProductScratch& ps, hipStream_t stream);

// One-triangle product for thin blocks (complex128, at most kTriMaxCols columns): the same
// product reading only the lower triangle of H, with partial sums in ps (tri_scratch_bytes).
// Returns hipErrorInvalidValue without launching when ps is too small; with ps.sk_need set it
// only raises *ps.sk_need to the bytes it needs.
constexpr int kTriMaxCols = 8;
// The solver's thin products (the Lanczos block) read one triangle from order kTriMinOrder and
// up to kTriSolverCols columns: measured at orders 2000 to 20000 it takes 0.5 to 0.75 of the
// full-read thin tile's time up to 3 columns, 0.7 to 0.95 at 4, 0.8 to 1.0 at 5, and longer
// than the thin tile from 6 columns.
constexpr int kTriSolverCols = 5;
constexpr int64_t kTriMinOrder = 2000;
size_t tri_scratch_bytes(int64_t n, int64_t ncols);
hipError_t launch_hemm_tri(const double* H, int64_t ldh, int64_t n, const double* X, int64_t ldx,
                           double* OUT, int64_t ldo, int64_t ncols, double alpha, double beta,
                           double gamma, const ProductScratch& ps, hipStream_t stream);
// The same product for real symmetric H and real X, OUT (T = double or float); leading
// dimensions count real elements.
template <typename T>
hipError_t launch_hemm_step_real(const T* H, int64_t ldh, int64_t n, const T* X, int64_t ldx,
                                 T* OUT, int64_t ldo, int64_t ncols, T alpha, T beta, T gamma,
                                 const ProductScratch& ps, hipStream_t stream);

// One product of one problem inside a grouped launch (fields as in launch_hemm_step; the
// last four are filled by the launcher).  Zero-column products are allowed and skipped.
template <typename T>
struct GroupDesc {
  const T* H;
  const T* X;
  T* OUT;
  int64_t ldh, ldx, ldo;
  int n, ncols;
  T alpha, beta, gamma;
  int tile_begin;    // first workgroup of this product in the main launch
  int ksplit;        // K slices per output tile (1: each tile is finished in place)
  int fix_begin;     // first workgroup of this product in the fixup launch (ksplit > 1)
  int64_t part_off;  // offset (values) of this product's partial sums in the scratch
};
constexpr int kMaxGroup = 16;
template <typename T>
struct GroupArgs {
  int count;
  T* partial;
  GroupDesc<T> d[kMaxGroup];
};
// Partial-sum scratch of K-sliced grouped products (owned by the batcher, fixed size).
struct GroupScratch {
  void* ptr = nullptr;
  size_t bytes = 0;
  int cus = 0;  // compute units of the device (0: every product stays in a grouped launch)
};
// Bytes the largest single K-sliced product can need; a scratch of at least this size lets the
// launchers run any group (in several launches when one does not fit).
size_t group_scratch_min_bytes();
// Grouped products.  Each product is computed exactly as it would be computed alone in a
// grouped launch: its K split (ksplit) is a function of its own order and width only, its tiles
// keep a fixed K order, and the slices of a split tile are added in slice order by a second
// (fixup) launch.  Results therefore do not depend on the grouping.  A product with few tiles
// is split along K so that a lone small product still occupies the whole device.  A product
// with more tiles than half the grouped launch's target (it fills the device by itself) runs
// on its own with the single-product schedule (data-parallel or stream-K, chosen from its
// shape and the device), using the group scratch for its partial sums when gs.cus is set.
template <typename T>
hipError_t launch_hemm_group(const GroupDesc<T>* descs, int count, const GroupScratch& gs,
                             hipStream_t stream);
// 3M products on planar complex64 H (Re plane, then Im plane at H + ldh * n).
hipError_t launch_hemm_step_3m(const float* H, int64_t ldh, int64_t n, const float* X,
                               int64_t ldx, float* OUT, int64_t ldo, int64_t ncols, float alpha,
                               float beta, float gamma, const ProductScratch& ps,
                               hipStream_t stream);
hipError_t launch_hemm_group_3m(const GroupDesc<float>* descs, int count, const GroupScratch& gs,
                                hipStream_t stream);
// 3M products on planar complex128 H (Re plane, then Im plane at H + ldh * n), FP64 MFMA.
hipError_t launch_hemm_step_3m_f64(const double* H, int64_t ldh, int64_t n, const double* X,
                                   int64_t ldx, double* OUT, int64_t ldo, int64_t ncols,
                                   double alpha, double beta, double gamma,
                                   const ProductScratch& ps, hipStream_t stream);
hipError_t launch_hemm_group_3m_f64(const GroupDesc<double>* descs, int count,
                                    const GroupScratch& gs, hipStream_t stream);
hipError_t launch_convert_c128_to_planar64(const double* src, int64_t lds, double* dst,
                                           int64_t ldd, int64_t n, hipStream_t stream);
hipError_t launch_convert_c128_to_planar32(const double* src, int64_t lds, float* dst, int64_t ldd,
                                           int64_t n, hipStream_t stream);

hipError_t launch_convert_c128_to_c64(const double* src, int64_t lds, float* dst, int64_t ldd,
                                      int64_t rows, int64_t cols, hipStream_t stream);
hipError_t launch_convert_c64_to_c128(const float* src, int64_t lds, double* dst, int64_t ldd,
                                      int64_t rows, int64_t cols, hipStream_t stream);

// Real float64 <-> float32 copies of an m x cols column-major block.
hipError_t launch_convert_f64_to_f32(const double* src, int64_t lds, float* dst, int64_t ldd,
                                     int64_t rows, int64_t cols, hipStream_t stream);
hipError_t launch_convert_f32_to_f64(const float* src, int64_t lds, double* dst, int64_t ldd,
                                     int64_t rows, int64_t cols, hipStream_t stream);

// Outer-loop helpers (loop_kernels.hip; the Cholesky factorisation in chol.hip), for double (complex128 / float64) and float (complex64
// / float32) vectors.  w = values per element: 2 for interleaved complex data, 1 for real data;
// leading dimensions count elements.  Scalars (Lanczos coefficients, residual norms) are double.
#define CHASE_LOOP_DECL(R)                                                                      \
  hipError_t launch_lanczos_step(const R* U, const R* Up, R* W, R* Un, int64_t n, int64_t ld,   \
                                 int64_t nv, const double* beta_prev, double* alpha_out,        \
                                 double* beta_out, hipStream_t s, int w = 2);                   \
  hipError_t launch_normalize(R* X, int64_t n, int64_t ld, int64_t cols, hipStream_t s,         \
                              int w = 2);                                                       \
  hipError_t launch_resid(const R* AV, const R* V, const R* lam, int64_t n, int64_t ld,         \
                          int64_t cols, double* out, hipStream_t s, int w = 2);                 \
  hipError_t launch_gather(const R* src, int64_t lds, R* dst, int64_t ldd, int64_t n,           \
                           const int* perm, int64_t cols, hipStream_t s, int w = 2);            \
  hipError_t launch_herm_sym(R* G, int64_t ld, int64_t m, hipStream_t s, int w = 2);            \
  hipError_t launch_add_diag(R* G, int64_t ld, int64_t m, double v, hipStream_t s, int w = 2);  \
  hipError_t launch_sum_slices(const R* P, int64_t m1, int64_t m2, int64_t stride, int p, R* G,  \
                              int64_t ldg, hipStream_t s, int w = 2);                           \
  hipError_t launch_gaussian(R* X, int64_t n, int64_t ld, int64_t cols, uint64_t seed,          \
                             hipStream_t s, int w = 2);                                         \
  hipError_t launch_potrf_upper(R* G, int64_t ld, int64_t m, int* info, hipStream_t s,          \
                                int w = 2);
CHASE_LOOP_DECL(double)
CHASE_LOOP_DECL(float)
// Interleaved complex64 H (ld lds) -> planar complex64 (Re plane, Im plane at dst + ldd * n).
hipError_t launch_split_planes_c64(const float* src, int64_t lds, float* dst, int64_t ldd,
                                   int64_t n, hipStream_t s);
#undef CHASE_LOOP_DECL

// ----------------------------------------------------------------------------- filter driver

// Algorithm 4 on an n x ncols block with sorted even degrees (validated by the caller).  The
// result ends in V.  scalars: the per-product (alpha, beta, gamma) in FP64.
// kind: 0 complex128 (4M), 1 complex64 interleaved (4M), 2 complex64 planar H (3M),
// 3 real data (T = double or float), 4 complex128 planar H (3M, FP64).
template <typename T>
hipError_t run_filter(const T* H, int64_t ldh, int64_t n, T* V, T* W, int64_t ld, int64_t ncols,
                      const int32_t* degrees, double b_sup, double mu_1, double mu_nevnex,
                      const ProductScratch& ps, hipStream_t stream, int64_t* matvecs_out,
                      int kind = 0);

// Continuous batching of filter products across concurrent solves: the products of every
// submitted filter call advance one per tick, each tick being one grouped launch per precision
// on the batcher's own stream.
class Batcher {
 public:
  explicit Batcher(int device);
  ~Batcher();
  bool ok() const { return ok_; }
  // Enqueue the products of one filter call; returns once all are launched, after making
  // `caller` wait for their completion.  fp64: complex128 data, else complex64.  `ready` and
  // `done` are events owned by the caller (reused across calls, destroyed only after the
  // caller's stream has drained).
  // kind: 0 complex128, 1 complex64 interleaved H, 2 complex64 planar H (3M).
  hipError_t run(int kind, const void* H, int64_t ldh, int64_t n, void* V, void* W, int64_t ld,
                 const std::vector<FilterProduct>& prods, hipStream_t caller, hipEvent_t ready,
                 hipEvent_t done);
  void counters(int64_t* launches, int64_t* products) const;
  // Device memory each batcher holds for its lifetime (the K-slice partial sums).
  static size_t scratch_bytes();

 private:
  struct Job;
  struct Impl;
  Impl* impl_ = nullptr;
  bool ok_ = false;
};

}  // namespace chase

struct chase_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  rocblas_handle blas = nullptr;
  chase::ProductScratch prod;
  std::string last_error;
  // device workspace, grown monotonically
  void* ws = nullptr;
  size_t ws_bytes = 0;
};

namespace chase {
int set_error(chase_ctx* ctx, int code, const std::string& msg);
int ensure_workspace(chase_ctx* ctx, size_t bytes);
int hip_ok(chase_ctx* ctx);  // hipSetDevice(ctx->device) with error reporting
class Batcher;
// chase_solve with an optional batcher for the filter products (serving).
int solve_with(chase_ctx* ctx, const chase_config* cfg, const void* H, int64_t ldh, void* V,
               int64_t ldv, double* ritzv, double* resid, chase_stats* stats, Batcher* batcher);
int check_config(chase_ctx* ctx, const chase_config* cfg);
// Argument checks of chase_filter / chase_hemm_step (messages go to ctx->last_error).
int check_product_args(chase_ctx* ctx, int precision, const void* H, int64_t ldh, int64_t n,
                       const void* X, int64_t ldx, const void* OUT, int64_t ldo, int64_t ncols);
int check_degrees(chase_ctx* ctx, const int32_t* degrees, int64_t ncols);
int check_bounds(chase_ctx* ctx, double b_sup, double mu_1, double mu_nevnex);
// Algorithm 4 in the given chase_precision (checked beforehand), products on `ps`.
hipError_t run_filter_precision(int precision, const void* H, int64_t ldh, int64_t n, void* V,
                                void* W, int64_t ld, int64_t ncols, const int32_t* degrees,
                                double b_sup, double mu_1, double mu_nevnex,
                                const ProductScratch& ps, hipStream_t stream);
// Layout of a solve's H and V elements: bytes per real scalar (8, or 4 for CHASE_FP32) and
// values per element (2 complex, 1 real symmetric).
inline int solve_scalar_bytes(const chase_config& c) { return c.precision == CHASE_FP32 ? 4 : 8; }
inline int solve_width(const chase_config& c) { return c.real_symmetric ? 1 : 2; }
inline size_t solve_elem_bytes(const chase_config& c) {
  return static_cast<size_t>(solve_scalar_bytes(c)) * solve_width(c);
}
// Gaussian start block for a solve's V in the solve's own element type.
hipError_t launch_start_block(void* V, const chase_config& c, uint64_t seed, hipStream_t s);
}  // namespace chase

#define CHASE_HIP_TRY(ctx, expr)                                                            \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return ::chase::set_error((ctx), CHASE_EDEVICE,                                       \
                                std::string(#expr) + ": " + hipGetErrorString(_e));         \
  } while (0)
