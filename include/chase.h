/*
 * chase.h -- C ABI of an MI355X (gfx950) implementation of ChASE, the Chebyshev Accelerated
 * Subspace iteration Eigensolver (Winkelmann, Springer, Di Napoli, arXiv:1805.10121).
 *
 * The library finds the nev smallest eigenpairs of a dense complex Hermitian matrix H of order n
 * with a search space of nev+nex vectors (Algorithm 1 of the paper).  Its hot path is the
 * Chebyshev filter (Algorithm 4, Eq. (7)), run as hand-written gfx950 kernels.
 *
 * Conventions shared by every call
 *   - Matrices are column-major.  "complex128" is two IEEE doubles (re, im) per element, the
 *     layout of C99 double complex / std::complex<double>; "complex64" is two floats.
 *   - "device" pointers are HIP device memory on the context's device; "host" pointers are
 *     ordinary host memory.  The caller owns every buffer it passes; the library never frees,
 *     reallocates or keeps them after the call returns, and never writes to H.
 *   - Every call returns a chase_status.  On a negative status a message is available from
 *     chase_last_error(ctx).  Argument checks are done before any device work is enqueued, so
 *     a CHASE_EINVAL return leaves every buffer untouched.
 *   - Work is ordered on the context's HIP stream.  chase_filter and the conversion calls only
 *     enqueue (they return before the GPU finishes); chase_solve and the sequence calls
 *     return after the GPU work has completed.
 *   - A context must not be used from two host threads at once.
 */
#ifndef CHASE_MI355X_H
#define CHASE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CHASE_OK = 0,
  CHASE_NOT_CONVERGED = 1,  /* maxIter reached: the current approximations are returned (Sec. 5.3) */
  CHASE_EINVAL = -1,        /* invalid argument; nothing was enqueued                            */
  CHASE_ENOMEM = -2,        /* device workspace could not be allocated                           */
  CHASE_EDEVICE = -3,       /* a HIP / rocBLAS / rocSOLVER call failed                           */
  CHASE_ENUMERIC = -4,      /* NaN/Inf, or orthonormalisation broke down even after fallback      */
  CHASE_EBUSY = -5          /* server: request does not fit the memory budget right now           */
} chase_status;

typedef enum {
  CHASE_FP64 = 0,   /* complex128 buffers, FP64 MFMA with FP64 accumulation                     */
  CHASE_FP32 = 1,   /* complex64 buffers, FP32 MFMA with FP32 accumulation.  chase_solve: the
                       whole solve in single precision (the paper's C / S instances, Sec. 5.1):
                       complex64 H and V, or float32 with real_symmetric = 1                   */
  CHASE_MIXED = 2,  /* chase_solve only: FP32 filter while a vector's relative residual exceeds
                       switch_resid, FP64 afterwards; everything outside the filter stays FP64 */
  CHASE_FP32_3M = 3, /* chase_filter / chase_hemm_step: H is "planar complex64" -- two real
                       n x n FP32 planes, Re H then Im H at an offset of ldh * n floats, each
                       column-major with leading dimension ldh -- and the products use three
                       real FP32 MFMA products per complex product (3M) with FP64 sums across
                       K stages; the blocks are complex64 as for CHASE_FP32 */
  CHASE_REAL_FP64 = 4, /* chase_filter / chase_hemm_step: real symmetric H and real blocks, all
                       float64 (the paper's real "D" instance, Sec. 5.1), FP64 MFMA            */
  CHASE_REAL_FP32 = 5, /* the same with float32 H and blocks, FP32 MFMA with FP32 accumulation */
  CHASE_FP64_3M = 6, /* chase_filter / chase_hemm_step: H is "planar complex128" -- two real
                       n x n float64 planes, Re H then Im H at an offset of ldh * n doubles --
                       and the products use three real FP64 MFMA products per complex product
                       (3M, 6 instead of 8 real flops per complex multiply-add) with FP64
                       accumulation; the blocks are complex128 as for CHASE_FP64 */
  CHASE_FP64_LOWER = 7 /* chase_hemm_step only, at most 8 columns: complex128 H of which only
                       the lower triangle and the diagonal are read (the Hermitian product of
                       Sec. 5.1.1 that uses one triangle; the upper triangle may hold anything),
                       FP64 arithmetic on the vector units; half the HBM bytes of a full read
                       for the thin blocks where the product is bound by reading H */
} chase_precision;

/*
 * Solver parameters.  The first block is Table 1 of the paper (Sec. 5.3) with its
 * double-precision defaults; chase_config_init fills them.  The second block holds settings the
 * paper leaves open.
 */
typedef struct chase_config {
  int64_t n;             /* order of H (Alg. 1 input A)                                          */
  int64_t nev;           /* wanted eigenpairs, 1 <= nev                                          */
  int64_t nex;           /* extra search vectors, nev + nex <= n                                 */
  int32_t approx;        /* 0: cold start (Lanczos DoS estimates, Alg. 6); 1: warm start from V
                            and ritzv (Sec. 3.3)                                     default 0   */
  double tol;            /* residual threshold (Alg. 1, Alg. 3)                      1e-10       */
  int32_t max_iter;      /* outer-loop cap (Sec. 5.3)                                25          */
  int32_t optim;         /* per-vector degrees (Alg. 5) instead of constant deg      0           */
  int32_t deg_extra;     /* DEGEXTRA of Alg. 5                                        2           */
  int32_t deg_max;       /* DEGMAX of Alg. 5                                          36          */
  int32_t deg;           /* initial / constant degree (Alg. 1), rounded up to even    20          */
  int32_t lanczos_iter;  /* k of Alg. 6                                               25          */
  int32_t num_lanczos;   /* n_vec of Alg. 6                                           4           */

  int32_t precision;     /* chase_precision: FP64, FP32 (single-precision solve) or MIXED  FP64  */
  double switch_resid;   /* MIXED: relative residual below which a vector is filtered in FP64
                                                                                      1e-6        */
  int32_t deg_max_fp32;  /* MIXED: DEGMAX for FP32-filtered vectors (Table 1 SP value) 18         */
  int32_t resid_relative;/* 1: converged iff Res <= tol * ||H||_est, where ||H||_est is the
                            largest |Ritz value| of the b_sup Lanczos run (a lower bound of
                            ||H||_2); 0: absolute Res <= tol as in the paper's experiments  1   */
  int32_t intersperse;   /* cold start: put Lanczos Ritz vectors below mu_{nev+nex} into the
                            leading columns of the start block (Alg. 6)               1           */
  double dos_sigma;      /* Gaussian width of the DoS (Sec. 4.2), on the [-1, 1] scale 0.25      */
  uint64_t seed;         /* seed of the counter-based generator for Lanczos start vectors   0    */
  const void* lanczos_start; /* optional device n x (1 + num_lanczos) block (ld = n) of Lanczos
                            start vectors in the element type of V; NULL: drawn from seed  NULL */
  int32_t have_mu;       /* cold start only: 1 = use mu_1 / mu_nevnex below instead of the DoS
                            estimates (Alg. 1 input "estimates mu_1 and mu_{nev+nex}")    0     */
  double mu_1, mu_nevnex;
  int32_t verbose;       /* 1: one line per outer iteration on stderr (locked pairs, largest
                            active residual, FP32 columns, elapsed time)                  0     */
  int32_t real_symmetric;/* 1: H is real symmetric and V real, float64 (float32 under CHASE_FP32)
                            (the paper's real instances); leading dimensions count real elements.
                            0: complex Hermitian complex128 (complex64 under CHASE_FP32)    0    */
  int32_t filter_3m;     /* complex128 data (FP64 and MIXED): 1 = the FP64 filter products and the
                            Rayleigh-Ritz product H Q use the 3M scheme (CHASE_FP64_3M) on a
                            planar copy of H made once per solve (16 n^2 bytes of workspace);
                            0 = the 4M scheme on H itself, no copy.  Solves run by the server
                            follow the same setting in their grouped products.            1     */
} chase_config;

/* Counters and timings of one solve (Sec. 6 reports iterations, matvecs and filter time). */
typedef struct chase_stats {
  int32_t status;          /* chase_status of the solve                                       */
  int32_t iterations;      /* outer-loop iterations                                           */
  int32_t nconv;           /* locked (converged) pairs                                        */
  int32_t fp32_iterations; /* iterations in which some columns were filtered in FP32          */
  int32_t qr_fallbacks;    /* Householder fallbacks taken by the orthonormalisation           */
  int32_t reserved;
  int64_t matvecs;         /* products of H with one vector, all phases                      */
  int64_t filter_matvecs;  /* sum over filter calls of the active degrees                    */
  double filter_flops;     /* 8 n^2 * filter_matvecs: algorithmic filter flops               */
  double filter_ms, lanczos_ms, ortho_ms, rr_ms, resid_ms, total_ms;
  double b_sup, mu_1, mu_nevnex, norm_est;
} chase_stats;

typedef struct chase_ctx chase_ctx;

/* Fill cfg with the Table 1 defaults for the given sizes.  No device work. */
void chase_config_init(chase_config* cfg, int64_t n, int64_t nev, int64_t nex);

/* The same with Table 1's single-precision defaults (tol 1e-5, deg_max 18, deg 10, k = 12) and
   precision = CHASE_FP32, for a solve on complex64 (or, with real_symmetric = 1, float32) data.
   No device work; a NULL cfg is ignored. */
void chase_config_init_fp32(chase_config* cfg, int64_t n, int64_t nev, int64_t nex);

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to order all work on, or
   NULL for a stream owned by the context.  Allocates a fixed partial-sum scratch for the
   stream-K schedule of the product kernel (two tile-sized slots per persistent workgroup:
   128 MiB on a 256-CU device) and a rocBLAS handle; the solver workspace comes later. */
int chase_create(chase_ctx** out, int device, void* hip_stream);
void chase_destroy(chase_ctx* ctx);

/* Text of the last error on this context ("" if none).  Valid until the next call on ctx. */
const char* chase_last_error(const chase_ctx* ctx);

/* Device bytes chase_solve will hold for cfg: the blocks, Lanczos vectors and small matrices,
   plus the FP32 copy of H that MIXED solves (4 w n^2 bytes) and single-precision complex solves
   (planar, 8 n^2 bytes) make; the caller's H itself is not counted.  No device work. */
size_t chase_workspace_bytes(const chase_config* cfg);

/*
 * The Chebyshev filter of Algorithm 4 with the scaled three-term recurrence of Eq. (7).
 *
 * For every column a of the n x ncols block V, replaces V[:, a] by p_{m_a}(H) V[:, a], where p_m
 * is the degree-m Chebyshev polynomial of Eq. (5) for the interval [mu_nevnex, b_sup] scaled so
 * that p_m(mu_1) = 1.  Product i of the recurrence (i = 1 .. max m) is one kernel launch
 * over the columns with m_a >= i (Alg. 4, its recurrence loop); the two buffers swap after every
 * product.  Because all m_a are even, every column's last product lands in the buffer that
 * held the input, so the result is returned in V and W is scratch (Sec. 4.1.3).
 *
 *   precision  CHASE_FP64: H, V, W are complex128.  CHASE_FP32: H, V, W are complex64 (use the
 *              conversion calls below to stage them); the recurrence coefficients are computed
 *              in FP64 and rounded to FP32 per launch.  CHASE_FP32_3M: planar complex64 H.
 *              CHASE_FP64_3M: planar complex128 H, complex128 V, W.
 *              CHASE_REAL_FP64 / CHASE_REAL_FP32: real symmetric H and real V, W (float64 /
 *              float32); leading dimensions count real elements.
 *   H          device, n x n, column-major, leading dimension ldh >= n, full Hermitian (or
 *              symmetric) storage (both triangles are read).  Read only.
 *   V          device, n x ncols, leading dimension ld >= n.  In: the block.  Out: the result.
 *   W          device, n x ncols, leading dimension ld, must not overlap V or H.  Scratch.
 *   degrees    host, ncols int32, sorted ascending, even, 2 <= m_a <= 64 (the sort of Alg. 1
 *              and the even rounding of Alg. 5 establish these properties).
 *   b_sup, mu_1, mu_nevnex   the spectral bounds Alg. 4 takes as input; need mu_1 < mu_nevnex < b_sup.
 * ncols == 0 is a no-op.  Enqueues only.
 */
int chase_filter(chase_ctx* ctx, int precision, const void* H, int64_t ldh, int64_t n, void* V,
                 void* W, int64_t ld, int64_t ncols, const int32_t* degrees, double b_sup,
                 double mu_1, double mu_nevnex);

/*
 * chase_filter for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same operation, arguments and result
 * as chase_filter (bitwise the same products), but it needs no context and allocates nothing:
 * no hipMalloc, hipFree or allocating library call.
 *
 *   device, hip_stream  the HIP device (made current by the call) and a hipStream_t on it to
 *              enqueue on (NULL: the device's null stream).
 *   precision .. mu_nevnex   as in chase_filter.
 *   err        host buffer of err_len bytes for an error message (may be NULL); "" on success.
 * The stream-K partial sums of the products live in a fixed 96 MiB device array that the library
 * holds on every GPU it runs on until the process ends.  The first call on a device (an empty
 * call, ncols = 0, is enough; make it before any graph capture) looks the array's address up.
 * A call whose products would need more than 96 MiB of partial sums -- on a 256-CU device only
 * CHASE_REAL_FP64 on more than 16 columns can -- returns CHASE_EINVAL with nothing enqueued.
 * Calls that overlap on one GPU share the array and race: order them on one stream.
 * Returns CHASE_OK, CHASE_EINVAL (argument errors, nothing enqueued) or CHASE_EDEVICE.
 */
int chase_filter_noalloc(int device, void* hip_stream, int precision, const void* H,
                         int64_t ldh, int64_t n, void* V, void* W, int64_t ld, int64_t ncols,
                         const int32_t* degrees, double b_sup, double mu_1, double mu_nevnex,
                         char* err, size_t err_len);

/*
 * One fused product of the filter (the kernel behind every launch of chase_filter):
 *     OUT[:, j] <- alpha * H X[:, j] + gamma * X[:, j] + beta * OUT[:, j],   j < ncols
 * With beta == 0 the old OUT is not read (it may hold NaN).  Also serves the other products of
 * the outer loop: H Q for Rayleigh-Ritz (Alg. 2) and the Lanczos block (Alg. 6).
 * X and OUT: device, n x ncols, leading dimensions ldx, ldo >= n; must not overlap each other
 * or H.  Types as in chase_filter; CHASE_FP64_LOWER as CHASE_FP64 but reading only the lower
 * triangle of H, for ncols <= 8 (CHASE_EINVAL above that, or when its partial sums, about
 * n^2 ncols / (4 S) bytes with S = 8, 4, 2 for 1-2, 3-5, 6-8 columns at large n, exceed the
 * context's product scratch of 128 MiB: orders above about 11500 at 8 columns, 20700 at 5,
 * 46000 at 2, 65000 at 1).  Results are bitwise reproducible.  Enqueues only.
 */
int chase_hemm_step(chase_ctx* ctx, int precision, const void* H, int64_t ldh, int64_t n,
                    const void* X, int64_t ldx, void* OUT, int64_t ldo, int64_t ncols,
                    double alpha, double beta, double gamma);

/* Precision staging of the mixed filter: dst = (complex64) src / (complex128) src on a
   rows x cols column-major block; planar32 writes the n x n matrix as the two FP32 planes of
   CHASE_FP32_3M (dst: 2 * ld_dst * n floats), planar64 as the two float64 planes of
   CHASE_FP64_3M (dst: 2 * ld_dst * n doubles).  Device pointers; enqueues only. */
int chase_convert_c128_to_planar32(chase_ctx* ctx, const void* src, int64_t ld_src, void* dst,
                                   int64_t ld_dst, int64_t n);
int chase_convert_c128_to_planar64(chase_ctx* ctx, const void* src, int64_t ld_src, void* dst,
                                   int64_t ld_dst, int64_t n);
int chase_convert_c128_to_c64(chase_ctx* ctx, const void* src, int64_t ld_src, void* dst,
                              int64_t ld_dst, int64_t rows, int64_t cols);
int chase_convert_c64_to_c128(chase_ctx* ctx, const void* src, int64_t ld_src, void* dst,
                              int64_t ld_dst, int64_t rows, int64_t cols);

/*
 * Algorithm 1: the nev smallest eigenpairs of H.
 *
 * Element type of H and V ("the solve's element type"): complex128 (precision FP64 or MIXED),
 * complex64 (FP32); with real_symmetric = 1 float64 or float32 instead.  Leading dimensions count
 * elements.  Ritz values, residuals and stats are double in every case.
 *
 *   H      device, n x n, ldh >= n, full Hermitian (symmetric) storage, read only.
 *   V      device, n x (nev+nex), ldv >= n.
 *          In, approx = 0: the random start block (Alg. 1 input V-hat).
 *          In, approx = 1: approximate eigenvectors, e.g. the previous solution in a sequence.
 *          Out: columns [0, nev) eigenvectors of ritzv[0..nev) (ascending), then the remaining
 *          nex Ritz vectors -- the warm start of the next problem.
 *   ritzv  host, nev+nex doubles.  In (approx = 1): previous eigenvalues; their min and max are
 *          mu_1 and mu_{nev+nex} (Sec. 3.3).  Out: Ritz values, ascending within the locked and
 *          the active parts.
 *   resid  host, nev+nex doubles.  Out: residual norms ||H v - lambda v||_2.
 *   stats  host, may be NULL.
 * Returns CHASE_OK, or CHASE_NOT_CONVERGED with the outputs filled when maxIter was reached.
 * Blocks until done.
 */
int chase_solve(chase_ctx* ctx, const chase_config* cfg, const void* H, int64_t ldh, void* V,
                int64_t ldv, double* ritzv, double* resid, chase_stats* stats);

/*
 * Sequences of correlated problems (Sec. 2, Sec. 6.1): the state -- the nev+nex vectors, the
 * Ritz values and the last degrees -- stays resident in device memory between problems.  The
 * first problem is solved cold, every later one warm (approx = 1) from the previous solution.
 */
typedef struct chase_seq chase_seq;
int chase_seq_create(chase_ctx* ctx, const chase_config* cfg, chase_seq** out);
/* Solve the next problem H (device, the solve's element type, ldh >= n).  ritzv / resid: host,
   nev+nex. */
int chase_seq_solve(chase_seq* seq, const void* H, int64_t ldh, double* ritzv, double* resid,
                    chase_stats* stats);
/* Borrowed device pointer to the current n x (nev+nex) vectors (valid until the next call). */
int chase_seq_vectors(chase_seq* seq, void** V, int64_t* ldv);
void chase_seq_destroy(chase_seq* seq);

/*
 * Serving: continuous batching of solves from many concurrent sequences of uneven order on one
 * device (the sequence setting of Sec. 2 and Sec. 6.1, served as requests arrive).
 *
 * Each request is one problem of a sequence identified by seq_id.  Problems of one sequence run
 * in submission order; the first is solved cold (cfg->approx as given), every later one is warm
 * started from the previous solution, which stays in device memory (the sequence state:
 * n x (nev+nex) vectors of the solve's element type and the Ritz values).  A request is started
 * when its sequence is idle and the device memory it needs -- the sequence state if new, plus
 * the growth of a worker's workspace (chase_workspace_bytes) -- fits in mem_budget_bytes beside
 * what is already held.  What is held includes the server's fixed allocations, charged at
 * creation: the batchers' partial-sum scratch and, per worker, the product scratch of its
 * context plus a 64 MiB allowance for its rocBLAS/rocSOLVER handle.  Up to `workers` requests
 * run at once, each on its own stream; the filter products of complex FP64 and MIXED requests
 * in flight are grouped into shared launches, one batcher (thread and stream) per size class
 * of n (below 3000, 6000, 12000, and the rest), so a small solve's products never wait behind
 * a much larger one's (real and FP32 requests run theirs on their worker's stream).  A request's
 * results are bitwise the same whatever else runs beside it.
 *
 * H: device, the solve's element type, n x n, ldh >= n, owned by the caller and kept valid and
 * unchanged until the request's ticket reports done.  n, nev and nex must stay the same within a
 * sequence.
 * Sequence states are held until chase_server_end_sequence or chase_server_destroy.
 */
typedef struct chase_server chase_server;
/* workers in [1, 64]; mem_budget_bytes above the fixed allocations (else CHASE_EINVAL).  Creates
   the batching threads and the workers. */
int chase_server_create(chase_server** out, int device, size_t mem_budget_bytes, int workers);
/* Queue one problem.  CHASE_EINVAL on a bad configuration or a size change inside a sequence;
   CHASE_EBUSY if the request alone needs more than the budget left beside the fixed
   allocations.  *ticket identifies it. */
int chase_server_submit(chase_server* s, uint64_t seq_id, const chase_config* cfg, const void* H,
                        int64_t ldh, uint64_t* ticket);
/* Poll (wait = 0) or wait (wait != 0) for a ticket.  When *done is set, ritzv / resid (host,
   nev+nex doubles), stats and latency_s (seconds from submit to completion) are filled (any may
   be NULL), the ticket is released, and the return value is the solve's chase_status. */
int chase_server_poll(chase_server* s, uint64_t ticket, int wait, int* done, double* ritzv,
                      double* resid, chase_stats* stats, double* latency_s);
/* Borrowed device pointer to an idle sequence's current vectors (CHASE_EINVAL if busy/unknown). */
int chase_server_vectors(chase_server* s, uint64_t seq_id, void** V, int64_t* ldv);
/* Release an idle sequence's state.  CHASE_EBUSY while it runs or has queued requests. */
int chase_server_end_sequence(chase_server* s, uint64_t seq_id);
/* Counters: grouped launches and products issued by the batchers, bytes held (fixed allocations,
   sequence states and worker workspaces). */
int chase_server_info(chase_server* s, int64_t* grouped_launches, int64_t* grouped_products,
                      size_t* bytes_in_use);
const char* chase_server_last_error(chase_server* s);
/* Finishes every queued request, then frees everything. */
void chase_server_destroy(chase_server* s);

#ifdef __cplusplus
}
#endif
#endif /* CHASE_MI355X_H */
