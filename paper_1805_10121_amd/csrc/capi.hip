// C ABI: contexts, configuration defaults, argument checking and the filter entry points.

#include <cmath>
#include <cstring>

#include "internal.h"

namespace chase {

int set_error(chase_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

int ensure_workspace(chase_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return CHASE_OK;
  if (ctx->ws) {
    CHASE_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    CHASE_HIP_TRY(ctx, hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  hipError_t e = hipMalloc(&ctx->ws, bytes);
  if (e != hipSuccess) {
    ctx->ws = nullptr;
    (void)hipGetLastError();
    return set_error(ctx, CHASE_ENOMEM,
                     "workspace allocation of " + std::to_string(bytes) + " bytes failed");
  }
  ctx->ws_bytes = bytes;
  return CHASE_OK;
}

static bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bbytes && pb < pa + abytes;
}

static size_t block_bytes(int64_t ld, int64_t rows, int64_t cols, size_t elem) {
  if (rows <= 0 || cols <= 0) return 0;
  return (static_cast<size_t>(cols - 1) * ld + rows) * elem;
}

int check_degrees(chase_ctx* ctx, const int32_t* degrees, int64_t ncols) {
  if (ncols > 0 && !degrees) return set_error(ctx, CHASE_EINVAL, "degrees is NULL");
  for (int64_t a = 0; a < ncols; ++a) {
    const int32_t m = degrees[a];
    if (m < 2 || m > 64 || (m & 1))
      return set_error(ctx, CHASE_EINVAL,
                       "degree " + std::to_string(m) + " at column " + std::to_string(a) +
                           " is not an even value in [2, 64]");
    if (a > 0 && m < degrees[a - 1])
      return set_error(ctx, CHASE_EINVAL, "degrees are not sorted ascending");
  }
  return CHASE_OK;
}

int check_bounds(chase_ctx* ctx, double b_sup, double mu_1, double mu_nevnex) {
  if (!std::isfinite(b_sup) || !std::isfinite(mu_1) || !std::isfinite(mu_nevnex))
    return set_error(ctx, CHASE_EINVAL, "spectral bounds must be finite");
  if (!(mu_1 < mu_nevnex && mu_nevnex < b_sup))
    return set_error(ctx, CHASE_EINVAL, "need mu_1 < mu_nevnex < b_sup");
  return CHASE_OK;
}

int check_product_args(chase_ctx* ctx, int precision, const void* H, int64_t ldh, int64_t n,
                       const void* X, int64_t ldx, const void* OUT, int64_t ldo, int64_t ncols) {
  if (precision < CHASE_FP64 || precision > CHASE_FP64_LOWER || precision == CHASE_MIXED)
    return set_error(ctx, CHASE_EINVAL,
                     "precision must be CHASE_FP64, CHASE_FP32, CHASE_FP32_3M, CHASE_REAL_FP64, "
                     "CHASE_REAL_FP32, CHASE_FP64_3M or (products only) CHASE_FP64_LOWER");
  if (n < 0 || ncols < 0) return set_error(ctx, CHASE_EINVAL, "negative size");
  if (n > 0x7fffffffLL || ncols > 0x7fffffffLL)
    return set_error(ctx, CHASE_EINVAL, "n and ncols must fit in int32");
  if (n == 0 || ncols == 0) return CHASE_OK;
  if (!H || !X || !OUT) return set_error(ctx, CHASE_EINVAL, "NULL buffer");
  if (ldh < n || ldx < n || ldo < n)
    return set_error(ctx, CHASE_EINVAL, "leading dimension smaller than n");
  const size_t elem =
      (precision == CHASE_FP64 || precision == CHASE_FP64_3M || precision == CHASE_FP64_LOWER) ? 16
      : precision == CHASE_REAL_FP32 ? 4
                                       : 8;
  // planar H: two ldh x n planes of floats (FP32_3M) or doubles (FP64_3M)
  const size_t hb = precision == CHASE_FP32_3M   ? static_cast<size_t>(ldh) * n * 8
                    : precision == CHASE_FP64_3M ? static_cast<size_t>(ldh) * n * 16
                                                 : block_bytes(ldh, n, n, elem);
  const size_t xb = block_bytes(ldx, n, ncols, elem);
  const size_t ob = block_bytes(ldo, n, ncols, elem);
  if (overlaps(X, xb, OUT, ob)) return set_error(ctx, CHASE_EINVAL, "X and OUT overlap");
  if (overlaps(H, hb, OUT, ob)) return set_error(ctx, CHASE_EINVAL, "H and OUT overlap");
  if (overlaps(H, hb, X, xb)) return set_error(ctx, CHASE_EINVAL, "H and X overlap");
  return CHASE_OK;
}

hipError_t run_filter_precision(int precision, const void* H, int64_t ldh, int64_t n, void* V,
                                void* W, int64_t ld, int64_t ncols, const int32_t* degrees,
                                double b_sup, double mu_1, double mu_nevnex,
                                const ProductScratch& ps, hipStream_t stream) {
  if (precision == CHASE_FP64 || precision == CHASE_REAL_FP64 || precision == CHASE_FP64_3M)
    return run_filter<double>(static_cast<const double*>(H), ldh, n, static_cast<double*>(V),
                              static_cast<double*>(W), ld, ncols, degrees, b_sup, mu_1, mu_nevnex,
                              ps, stream, nullptr,
                              precision == CHASE_REAL_FP64 ? 3 : precision == CHASE_FP64_3M ? 4 : 0);
  if (precision == CHASE_REAL_FP32)
    return run_filter<float>(static_cast<const float*>(H), ldh, n, static_cast<float*>(V),
                             static_cast<float*>(W), ld, ncols, degrees, b_sup, mu_1, mu_nevnex,
                             ps, stream, nullptr, 3);
  return run_filter<float>(static_cast<const float*>(H), ldh, n, static_cast<float*>(V),
                           static_cast<float*>(W), ld, ncols, degrees, b_sup, mu_1, mu_nevnex, ps,
                           stream, nullptr, precision == CHASE_FP32_3M ? 2 : 1);
}

}  // namespace chase

using namespace chase;

extern "C" {

void chase_config_init(chase_config* cfg, int64_t n, int64_t nev, int64_t nex) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->n = n;
  cfg->nev = nev;
  cfg->nex = nex;
  // Table 1 (double precision)
  cfg->approx = 0;
  cfg->tol = 1e-10;
  cfg->max_iter = 25;
  cfg->optim = 0;
  cfg->deg_extra = 2;
  cfg->deg_max = 36;
  cfg->deg = 20;
  cfg->lanczos_iter = 25;
  cfg->num_lanczos = 4;
  // settings the paper leaves open
  cfg->precision = CHASE_FP64;
  cfg->switch_resid = 1e-6;
  cfg->deg_max_fp32 = 18;
  cfg->resid_relative = 1;
  cfg->intersperse = 1;
  cfg->dos_sigma = 0.25;
  cfg->seed = 0;
  cfg->lanczos_start = nullptr;
  cfg->have_mu = 0;
  cfg->mu_1 = 0.0;
  cfg->mu_nevnex = 0.0;
  cfg->verbose = 0;
  cfg->real_symmetric = 0;
  cfg->filter_3m = 1;
}

void chase_config_init_fp32(chase_config* cfg, int64_t n, int64_t nev, int64_t nex) {
  if (!cfg) return;
  chase_config_init(cfg, n, nev, nex);
  // Table 1, single-precision values
  cfg->tol = 1e-5;
  cfg->deg_max = 18;
  cfg->deg = 10;
  cfg->lanczos_iter = 12;
  cfg->precision = CHASE_FP32;
}

int chase_create(chase_ctx** out, int device, void* hip_stream) {
  if (!out) return CHASE_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return CHASE_EDEVICE;
  }
  chase_ctx* ctx = new chase_ctx();
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return CHASE_EDEVICE;
  }
  if (hip_stream) {
    ctx->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreate(&ctx->stream) != hipSuccess) {
      delete ctx;
      return CHASE_EDEVICE;
    }
    ctx->own_stream = true;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus <= 0) {
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return CHASE_EDEVICE;
  }
  ctx->prod.cus = cus;
  ctx->prod.bytes = product_scratch_bytes(cus);
  if (hipMalloc(&ctx->prod.ptr, ctx->prod.bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return CHASE_ENOMEM;
  }
  // rocBLAS may pick kernels that add partial results with atomics (summation order then
  // depends on timing); they are refused so that results are bitwise reproducible, also when
  // other work shares the device.
  if (rocblas_create_handle(&ctx->blas) != rocblas_status_success ||
      rocblas_set_stream(ctx->blas, ctx->stream) != rocblas_status_success ||
      rocblas_set_atomics_mode(ctx->blas, rocblas_atomics_not_allowed) != rocblas_status_success) {
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    (void)hipFree(ctx->prod.ptr);
    delete ctx;
    return CHASE_EDEVICE;
  }
  *out = ctx;
  return CHASE_OK;
}

void chase_destroy(chase_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->prod.ptr) (void)hipFree(ctx->prod.ptr);
  if (ctx->blas) rocblas_destroy_handle(ctx->blas);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char* chase_last_error(const chase_ctx* ctx) {
  return ctx ? ctx->last_error.c_str() : "NULL context";
}

int chase_filter(chase_ctx* ctx, int precision, const void* H, int64_t ldh, int64_t n, void* V,
                 void* W, int64_t ld, int64_t ncols, const int32_t* degrees, double b_sup,
                 double mu_1, double mu_nevnex) {
  if (!ctx) return CHASE_EINVAL;
  ctx->last_error.clear();
  if (precision == CHASE_FP64_LOWER)
    return set_error(ctx, CHASE_EINVAL, "CHASE_FP64_LOWER applies to chase_hemm_step only");
  int rc = check_product_args(ctx, precision, H, ldh, n, V, ld, W, ld, ncols);
  if (rc) return rc;
  if (n == 0 || ncols == 0) return CHASE_OK;
  if ((rc = check_degrees(ctx, degrees, ncols))) return rc;
  if ((rc = check_bounds(ctx, b_sup, mu_1, mu_nevnex))) return rc;
  CHASE_HIP_TRY(ctx, hipSetDevice(ctx->device));
  const hipError_t e = run_filter_precision(precision, H, ldh, n, V, W, ld, ncols, degrees, b_sup,
                                            mu_1, mu_nevnex, ctx->prod, ctx->stream);
  if (e != hipSuccess)
    return set_error(ctx, CHASE_EDEVICE, std::string("filter launch: ") + hipGetErrorString(e));
  return CHASE_OK;
}

int chase_hemm_step(chase_ctx* ctx, int precision, const void* H, int64_t ldh, int64_t n,
                    const void* X, int64_t ldx, void* OUT, int64_t ldo, int64_t ncols,
                    double alpha, double beta, double gamma) {
  if (!ctx) return CHASE_EINVAL;
  ctx->last_error.clear();
  int rc = check_product_args(ctx, precision, H, ldh, n, X, ldx, OUT, ldo, ncols);
  if (rc) return rc;
  if (!std::isfinite(alpha) || !std::isfinite(beta) || !std::isfinite(gamma))
    return set_error(ctx, CHASE_EINVAL, "non-finite coefficient");
  if (n == 0 || ncols == 0) return CHASE_OK;
  CHASE_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipError_t e;
  if (precision == CHASE_FP64_LOWER) {
    if (ncols > kTriMaxCols)
      return set_error(ctx, CHASE_EINVAL, "CHASE_FP64_LOWER takes at most 8 columns");
    if (tri_scratch_bytes(n, ncols) > ctx->prod.bytes)
      return set_error(ctx, CHASE_EINVAL,
                       "CHASE_FP64_LOWER at this order and width needs " +
                           std::to_string(tri_scratch_bytes(n, ncols)) +
                           " bytes of partial sums; the context's scratch holds " +
                           std::to_string(ctx->prod.bytes));
  }
  if (precision == CHASE_FP64_LOWER)
    e = launch_hemm_tri(static_cast<const double*>(H), ldh, n, static_cast<const double*>(X), ldx,
                        static_cast<double*>(OUT), ldo, ncols, alpha, beta, gamma, ctx->prod,
                        ctx->stream);
  else if (precision == CHASE_FP64)
    e = launch_hemm_step<double>(static_cast<const double*>(H), ldh, n,
                                 static_cast<const double*>(X), ldx, static_cast<double*>(OUT),
                                 ldo, ncols, alpha, beta, gamma, ctx->prod, ctx->stream);
  else if (precision == CHASE_REAL_FP64)
    e = launch_hemm_step_real<double>(static_cast<const double*>(H), ldh, n,
                                      static_cast<const double*>(X), ldx,
                                      static_cast<double*>(OUT), ldo, ncols, alpha, beta, gamma,
                                      ctx->prod, ctx->stream);
  else if (precision == CHASE_REAL_FP32)
    e = launch_hemm_step_real<float>(static_cast<const float*>(H), ldh, n,
                                     static_cast<const float*>(X), ldx, static_cast<float*>(OUT),
                                     ldo, ncols, static_cast<float>(alpha),
                                     static_cast<float>(beta), static_cast<float>(gamma),
                                     ctx->prod, ctx->stream);
  else if (precision == CHASE_FP64_3M)
    e = launch_hemm_step_3m_f64(static_cast<const double*>(H), ldh, n,
                                static_cast<const double*>(X), ldx, static_cast<double*>(OUT), ldo,
                                ncols, alpha, beta, gamma, ctx->prod, ctx->stream);
  else if (precision == CHASE_FP32_3M)
    e = launch_hemm_step_3m(static_cast<const float*>(H), ldh, n, static_cast<const float*>(X), ldx,
                            static_cast<float*>(OUT), ldo, ncols, static_cast<float>(alpha),
                            static_cast<float>(beta), static_cast<float>(gamma), ctx->prod,
                            ctx->stream);
  else
    e = launch_hemm_step<float>(static_cast<const float*>(H), ldh, n,
                                static_cast<const float*>(X), ldx, static_cast<float*>(OUT), ldo,
                                ncols, static_cast<float>(alpha), static_cast<float>(beta),
                                static_cast<float>(gamma), ctx->prod, ctx->stream);
  if (e != hipSuccess)
    return set_error(ctx, CHASE_EDEVICE, std::string("product launch: ") + hipGetErrorString(e));
  return CHASE_OK;
}

static int convert_common(chase_ctx* ctx, const void* src, int64_t ld_src, void* dst,
                          int64_t ld_dst, int64_t rows, int64_t cols, size_t se, size_t de) {
  if (!ctx) return CHASE_EINVAL;
  ctx->last_error.clear();
  if (rows < 0 || cols < 0) return set_error(ctx, CHASE_EINVAL, "negative size");
  if (rows == 0 || cols == 0) return CHASE_OK;
  if (!src || !dst) return set_error(ctx, CHASE_EINVAL, "NULL buffer");
  if (ld_src < rows || ld_dst < rows)
    return set_error(ctx, CHASE_EINVAL, "leading dimension smaller than rows");
  if (overlaps(src, block_bytes(ld_src, rows, cols, se), dst, block_bytes(ld_dst, rows, cols, de)))
    return set_error(ctx, CHASE_EINVAL, "src and dst overlap");
  return CHASE_OK;
}

int chase_convert_c128_to_c64(chase_ctx* ctx, const void* src, int64_t ld_src, void* dst,
                              int64_t ld_dst, int64_t rows, int64_t cols) {
  int rc = convert_common(ctx, src, ld_src, dst, ld_dst, rows, cols, 16, 8);
  if (rc || rows == 0 || cols == 0) return rc;
  CHASE_HIP_TRY(ctx, hipSetDevice(ctx->device));
  CHASE_HIP_TRY(ctx, launch_convert_c128_to_c64(static_cast<const double*>(src), ld_src,
                                                static_cast<float*>(dst), ld_dst, rows, cols,
                                                ctx->stream));
  return CHASE_OK;
}

int chase_convert_c128_to_planar32(chase_ctx* ctx, const void* src, int64_t ld_src, void* dst,
                                   int64_t ld_dst, int64_t n) {
  if (!ctx) return CHASE_EINVAL;
  ctx->last_error.clear();
  if (n < 0) return set_error(ctx, CHASE_EINVAL, "negative size");
  if (n == 0) return CHASE_OK;
  if (!src || !dst) return set_error(ctx, CHASE_EINVAL, "NULL buffer");
  if (ld_src < n || ld_dst < n) return set_error(ctx, CHASE_EINVAL, "leading dimension < n");
  if (overlaps(src, block_bytes(ld_src, n, n, 16), dst, static_cast<size_t>(ld_dst) * n * 8))
    return set_error(ctx, CHASE_EINVAL, "src and dst overlap");
  CHASE_HIP_TRY(ctx, hipSetDevice(ctx->device));
  CHASE_HIP_TRY(ctx, launch_convert_c128_to_planar32(static_cast<const double*>(src), ld_src,
                                                     static_cast<float*>(dst), ld_dst, n,
                                                     ctx->stream));
  return CHASE_OK;
}

int chase_convert_c128_to_planar64(chase_ctx* ctx, const void* src, int64_t ld_src, void* dst,
                                   int64_t ld_dst, int64_t n) {
  if (!ctx) return CHASE_EINVAL;
  ctx->last_error.clear();
  if (n < 0) return set_error(ctx, CHASE_EINVAL, "negative size");
  if (n == 0) return CHASE_OK;
  if (!src || !dst) return set_error(ctx, CHASE_EINVAL, "NULL buffer");
  if (ld_src < n || ld_dst < n) return set_error(ctx, CHASE_EINVAL, "leading dimension < n");
  if (overlaps(src, block_bytes(ld_src, n, n, 16), dst, static_cast<size_t>(ld_dst) * n * 16))
    return set_error(ctx, CHASE_EINVAL, "src and dst overlap");
  CHASE_HIP_TRY(ctx, hipSetDevice(ctx->device));
  CHASE_HIP_TRY(ctx, launch_convert_c128_to_planar64(static_cast<const double*>(src), ld_src,
                                                     static_cast<double*>(dst), ld_dst, n,
                                                     ctx->stream));
  return CHASE_OK;
}

int chase_convert_c64_to_c128(chase_ctx* ctx, const void* src, int64_t ld_src, void* dst,
                              int64_t ld_dst, int64_t rows, int64_t cols) {
  int rc = convert_common(ctx, src, ld_src, dst, ld_dst, rows, cols, 8, 16);
  if (rc || rows == 0 || cols == 0) return rc;
  CHASE_HIP_TRY(ctx, hipSetDevice(ctx->device));
  CHASE_HIP_TRY(ctx, launch_convert_c64_to_c128(static_cast<const float*>(src), ld_src,
                                                static_cast<double*>(dst), ld_dst, rows, cols,
                                                ctx->stream));
  return CHASE_OK;
}

}  // extern "C"
