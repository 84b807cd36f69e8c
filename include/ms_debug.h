/*
 * ms_debug.h -- kernel-level entry points of the same library, exported for
 * unit tests of the building blocks behind ms.h (GEMM, LU solve, slice
 * eigensolver).  Same conventions as ms.h: device pointers, row-major,
 * interleaved complex, asynchronous on the context stream, numerical status
 * via ms_ctx_sync.  Not needed by users of the transport path.
 */
#ifndef MS_DEBUG_H
#define MS_DEBUG_H

#include "ms.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C = alpha op(A) op(B) + beta C for one M x N x K product.  op codes:
 * 0 = none, 1 = transpose, 2 = conjugate transpose.  prec = MS_PREC_FP64:
 * A, B, C complex128.  prec = MS_PREC_FP32_MFMA: A, B complex64, C complex128
 * (FP32 MFMA products, FP32 accumulation within 16-deep K-slabs summed in FP64).
 * alpha/beta: {re, im} host pairs. */
ms_status ms_debug_gemm(ms_ctx ctx, int op_a, int op_b, int64_t m, int64_t n, int64_t k, const void* a,
                        int64_t lda, const void* b, int64_t ldb, void* c, int64_t ldc, const double* alpha,
                        const double* beta, ms_prec prec);

/* Batched form of ms_debug_gemm: C[i] = alpha op(A[i]) op(B[i]) + beta C[i] for
 * i < batch, with element strides s_a, s_b, s_c between consecutive matrices
 * (0 = the same matrix for every i). */
ms_status ms_debug_gemm_batched(ms_ctx ctx, int op_a, int op_b, int64_t m, int64_t n, int64_t k, const void* a,
                                int64_t lda, int64_t s_a, const void* b, int64_t ldb, int64_t s_b, void* c,
                                int64_t ldc, int64_t s_c, int64_t batch, const double* alpha, const double* beta,
                                ms_prec prec);

/* The fused fold's interface product for `batch` energies sharing one overlap O:
 *   W[b] = A[b] [C-_b | C+_b with its diagonal set to 0],
 *   C-_b[m][j] = O[j][m] (kp_b[j] - kq_b[m]),  C+_b[m][j] = O[j][m] (kp_b[j] + kq_b[m])
 * (O^T K_p -+ K_q O^T, the operands of Phi_A and Phi_B in the star product of a slice
 * interface with the accumulated right part).  A [batch][n][n] (complex128, or complex64
 * with prec = MS_PREC_FP32_MFMA), O [n][n] complex128, kp, kq [batch][n] complex128 (entry b
 * at kp + b n), W [batch][n][2n] complex128.  The B operand is generated in FP64 from O, kp,
 * kq while it is staged and rounded to the product's type. */
ms_status ms_debug_iface_product(ms_ctx ctx, int64_t n, int64_t batch, const void* a, const void* o,
                                 const void* kp, const void* kq, void* w, ms_prec prec);

/* The same product with the fold's fused epilogue: m [batch][n][2n] c128 receives
 *   m[i][j]     = C+_ij + (A C-)_ij,
 *   m[i][n + j] = C-_ij + (A C+')_ij + rho_ij C+_jj,   rho_ij = pq_i kq_i y_ij pq_j / kq_j,
 * with C+-_ij = O_ji (kp_j +- kq_i), C+' = C+ without its diagonal; y [batch][n][n] c128,
 * pq [batch][n] c128. */
ms_status ms_debug_iface_fused(ms_ctx ctx, int64_t n, int64_t batch, const void* a, const void* o, const void* kp,
                               const void* kq, const void* y, const void* pq, void* m, ms_prec prec);

/* Eigenpairs of `batch` complex pencils A x = lam B x (n x n each, complex128, not modified) by
 * the library's QZ iteration: alpha, beta [batch][n] complex128 with lam = alpha / beta (beta
 * real >= 0; beta = 0 for an infinite eigenvalue), x [batch][n][n] right eigenvectors as unit
 * 2-norm columns, status [batch] int32 (MS_ERR_NOCONV if the iteration did not converge). */
ms_status ms_debug_qz(ms_ctx ctx, int64_t n, int64_t batch, const void* a, const void* b, void* alpha, void* beta,
                      void* x, int32_t* status);

/* For each of `batch` row-major n x (n + nrhs) complex128 matrices [A | B]
 * (batch stride n*(n+nrhs)), factor A with partial pivoting (in place) and
 * write X = A^-1 B to x (n x nrhs per matrix, batch stride n*nrhs).
 * status [batch] int32 device: MS_ERR_SINGULAR on a zero pivot. */
ms_status ms_debug_lu_solve(ms_ctx ctx, int64_t n, int64_t nrhs, int64_t batch, void* aug, void* x,
                            int32_t* status);

/* Eigenpairs of `batch` Hermitian n x n complex128 matrices h (not modified),
 * with the positivity shifts c [batch] f64 (h + c I must be positive definite):
 * eps [batch][n] ascending, u [batch][n][n] unit eigenvectors as columns. */
ms_status ms_debug_eigh(ms_ctx ctx, int64_t n, int64_t batch, const void* h, const double* shift,
                        double* eps, void* u);

/* Kernel timing with HIP events for the launches of the categories whose bit
 * is set in `mask` (0 stops recording).  GEMM launches pass their events to
 * hipExtLaunchKernel, so they measure the kernel's own execution; the other
 * kernels are bracketed by events recorded on the stream around the launch.
 * Categories, bit 0 upwards: "iface_gemm" (interface product of the fused
 * fold), "lu_panel", "lu_swap", "lu_update" (rank-128 trailing update),
 * "trsm", "jacobi", "prep_gemm", "elem", "other", "lu_inner" (updates inside
 * an outer LU panel and the U12 product).  ms_debug_profile_read waits for
 * the streams and returns, for the launches recorded since the previous read
 * of that category: summed duration (ms), launch count, and the algorithmic
 * flops and bytes the launches were sized for (GEMM: 8 M N K; bytes: operands
 * read once plus C written, read too when beta != 0). */
ms_status ms_debug_profile(ms_ctx ctx, uint32_t mask);
ms_status ms_debug_profile_read(ms_ctx ctx, const char* category, double* total_ms, int64_t* launches,
                                double* flops, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* MS_DEBUG_H */
