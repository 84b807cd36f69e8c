// Kernel-level entry points for unit tests (include/ms_debug.h).
#include <algorithm>
#include <cmath>

#include "../../include/ms_debug.h"
#include "elem.h"
#include "ms_internal.h"

using namespace ms;

namespace {
__global__ void k_add_shift(int n, const double* shift, double2* W) {
  const int64_t b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) W[b * (int64_t)n * n + (int64_t)i * n + i].x += shift[b];
}
}  // namespace

extern "C" {

ms_status ms_debug_gemm(ms_ctx ctx, int op_a, int op_b, int64_t m, int64_t n, int64_t k, const void* a, int64_t lda,
                        const void* b, int64_t ldb, void* c, int64_t ldc, const double* alpha, const double* beta,
                        ms_prec prec) {
  if (!ctx) return MS_ERR_ARG;
  if (!a || !b || !c || !alpha || !beta) return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (op_a < 0 || op_a > 2 || op_b < 0 || op_b > 2) return fail(ctx, MS_ERR_ARG, "op codes are 0, 1, 2");
  if (m <= 0 || n <= 0 || k < 0 || m > (1 << 30) || n > (1 << 30) || k > (1 << 30))
    return fail(ctx, MS_ERR_ARG, "bad sizes");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  GemmArgs g;
  g.M = (int)m; g.N = (int)n; g.K = (int)k;
  g.opA = op_a; g.opB = op_b;
  g.A = a; g.lda = lda; g.B = b; g.ldb = ldb;
  g.C = static_cast<double2*>(c); g.ldc = ldc;
  g.alpha = make_double2(alpha[0], alpha[1]);
  g.beta = make_double2(beta[0], beta[1]);
  if (prec == MS_PREC_FP64) return zgemm(ctx, g);
  if (prec == MS_PREC_FP32_MFMA) return cgemm32(ctx, g);
  return fail(ctx, MS_ERR_ARG, "unknown precision");
}

ms_status ms_debug_gemm_batched(ms_ctx ctx, int op_a, int op_b, int64_t m, int64_t n, int64_t k, const void* a,
                                int64_t lda, int64_t s_a, const void* b, int64_t ldb, int64_t s_b, void* c,
                                int64_t ldc, int64_t s_c, int64_t batch, const double* alpha, const double* beta,
                                ms_prec prec) {
  if (!ctx) return MS_ERR_ARG;
  if (!a || !b || !c || !alpha || !beta) return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (op_a < 0 || op_a > 2 || op_b < 0 || op_b > 2) return fail(ctx, MS_ERR_ARG, "op codes are 0, 1, 2");
  if (m <= 0 || n <= 0 || k < 0 || batch <= 0 || m > (1 << 30) || n > (1 << 30) || k > (1 << 30) ||
      batch > (1 << 20))
    return fail(ctx, MS_ERR_ARG, "bad sizes");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  GemmArgs g;
  g.M = (int)m; g.N = (int)n; g.K = (int)k;
  g.opA = op_a; g.opB = op_b;
  g.A = a; g.lda = lda; g.sA = s_a;
  g.B = b; g.ldb = ldb; g.sB = s_b;
  g.C = static_cast<double2*>(c); g.ldc = ldc; g.sC = s_c;
  g.batch = (int)batch;
  g.alpha = make_double2(alpha[0], alpha[1]);
  g.beta = make_double2(beta[0], beta[1]);
  if (prec == MS_PREC_FP64) return zgemm(ctx, g);
  if (prec == MS_PREC_FP32_MFMA) return cgemm32(ctx, g);
  return fail(ctx, MS_ERR_ARG, "unknown precision");
}

ms_status ms_debug_iface_product(ms_ctx ctx, int64_t n, int64_t batch, const void* a, const void* o,
                                 const void* kp, const void* kq, void* w, ms_prec prec) {
  if (!ctx) return MS_ERR_ARG;
  if (!a || !o || !kp || !kq || !w) return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (n <= 0 || batch <= 0 || n > 4096 || batch > 65535) return fail(ctx, MS_ERR_ARG, "bad sizes");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  GemmArgs g;
  g.M = (int)n; g.N = 2 * (int)n; g.K = (int)n;
  g.A = a; g.lda = n; g.sA = n * n; g.opA = OP_N;
  g.B = o; g.ldb = n; g.sB = 0; g.opB = OP_T;
  g.C = static_cast<double2*>(w); g.ldc = 2 * n; g.sC = 2 * n * n;
  g.batch = (int)batch;
  g.kp = static_cast<const double2*>(kp);
  g.kq = static_cast<const double2*>(kq);
  g.sk = n;
  g.prof = PC_IFACE_GEMM;
  if (prec == MS_PREC_FP64) return zgemm(ctx, g);
  if (prec == MS_PREC_FP32_MFMA) return cgemm32(ctx, g);
  return fail(ctx, MS_ERR_ARG, "unknown precision");
}

ms_status ms_debug_iface_fused(ms_ctx ctx, int64_t n, int64_t batch, const void* a, const void* o, const void* kp,
                               const void* kq, const void* y, const void* pq, void* m, ms_prec prec) {
  if (!ctx) return MS_ERR_ARG;
  if (!a || !o || !kp || !kq || !y || !pq || !m) return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (n <= 0 || batch <= 0 || n > 4096 || batch > 65535) return fail(ctx, MS_ERR_ARG, "bad sizes");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  GemmArgs g;
  g.M = (int)n; g.N = 2 * (int)n; g.K = (int)n;
  g.A = a; g.lda = n; g.sA = n * n; g.opA = OP_N;
  g.B = o; g.ldb = n; g.sB = 0; g.opB = OP_T;
  g.C = static_cast<double2*>(m); g.ldc = 2 * n; g.sC = 2 * n * n;
  g.batch = (int)batch;
  g.kp = static_cast<const double2*>(kp);
  g.kq = static_cast<const double2*>(kq);
  g.sk = n;
  g.ey = static_cast<const double2*>(y);
  g.eldy = n;
  g.esy = n * n;
  g.epq = static_cast<const double2*>(pq);
  g.prof = PC_IFACE_GEMM;
  if (prec == MS_PREC_FP64) return zgemm(ctx, g);
  if (prec == MS_PREC_FP32_MFMA) return cgemm32(ctx, g);
  return fail(ctx, MS_ERR_ARG, "unknown precision");
}

ms_status ms_debug_qz(ms_ctx ctx, int64_t n, int64_t batch, const void* a, const void* b, void* alpha, void* beta,
                      void* x, int32_t* status) {
  if (!ctx) return MS_ERR_ARG;
  if (!a || !b || !alpha || !beta || !x || !status) return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (n < 2 || batch <= 0 || n > 4096 || batch > 65535) return fail(ctx, MS_ERR_ARG, "bad sizes");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  const size_t bytes = (size_t)batch * n * n * sizeof(double2);
  void *A, *B, *V, *Y;
  MS_TRY(workspace(ctx, 60, bytes, &A));
  MS_TRY(workspace(ctx, 61, bytes, &B));
  MS_TRY(workspace(ctx, 62, bytes, &V));
  MS_TRY(workspace(ctx, 63, bytes, &Y));
  MS_HIP(ctx, hipMemcpyAsync(A, a, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(B, b, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  MS_TRY(launch_fill_i32(ctx, batch, status, 0));
  return qz_eig(ctx, (int)n, (int)batch, static_cast<double2*>(A), static_cast<double2*>(B), static_cast<double2*>(V),
                static_cast<double2*>(Y), static_cast<double2*>(alpha), static_cast<double2*>(beta),
                static_cast<double2*>(x), status);
}

ms_status ms_debug_lu_solve(ms_ctx ctx, int64_t n, int64_t nrhs, int64_t batch, void* aug, void* x, int32_t* status) {
  if (!ctx) return MS_ERR_ARG;
  if (!aug || !x || !status) return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (n <= 0 || nrhs <= 0 || batch <= 0) return fail(ctx, MS_ERR_ARG, "bad sizes");
  if (n > 4096 || batch > 65535) return fail(ctx, MS_ERR_UNSUPPORTED, "size beyond the supported limits");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  void* piv = nullptr;
  MS_TRY(workspace(ctx, 13, (size_t)batch * n * sizeof(int32_t), &piv));
  MS_HIP(ctx, hipMemsetAsync(status, 0, batch * sizeof(int32_t), ctx->stream));
  const int ncols = (int)(n + nrhs);
  double2* A = static_cast<double2*>(aug);
  MS_TRY(getrf_aug(ctx, A, (int)n, ncols, n * ncols, (int)batch, (int32_t*)piv, status, 1));
  return trsm_upper_aug(ctx, A, (int)n, ncols, n * ncols, (int)batch, static_cast<double2*>(x), nrhs, n * nrhs, status,
                        1);
}

ms_status ms_debug_eigh(ms_ctx ctx, int64_t n, int64_t batch, const void* h, const double* shift, double* eps,
                        void* u) {
  if (!ctx) return MS_ERR_ARG;
  if (!h || !shift || !eps || !u) return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (n <= 0 || batch <= 0) return fail(ctx, MS_ERR_ARG, "bad sizes");
  if (n > 3000 || batch > 65535) return fail(ctx, MS_ERR_UNSUPPORTED, "size beyond the supported limits");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t nn = n * n;
  void* W = nullptr;
  void* Z = nullptr;
  MS_TRY(workspace(ctx, 2, (size_t)batch * nn * sizeof(double2), &W));
  MS_TRY(workspace(ctx, 20, (size_t)batch * nn * sizeof(double2), &Z));
  MS_HIP(ctx, hipMemcpyAsync(W, h, (size_t)batch * nn * sizeof(double2), hipMemcpyDeviceToDevice, ctx->stream));
  hipLaunchKernelGGL(k_add_shift, dim3((unsigned)((n + 255) / 256), (unsigned)batch), dim3(256), 0, ctx->stream, (int)n,
                     shift, static_cast<double2*>(W));
  MS_TRY(check_launch(ctx, "add shift"));
  return jacobi_eigh(ctx, (int)n, (int)batch, static_cast<double2*>(W), static_cast<const double2*>(h),
                     static_cast<double2*>(Z), eps, n, static_cast<double2*>(u), nn, ctx->d_status);
}

}  // extern "C"
