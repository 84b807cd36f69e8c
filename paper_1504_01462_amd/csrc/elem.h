// Launchers of the per-energy elementwise kernels (elem.hip).
#pragma once
#include "ms_internal.h"

namespace ms {

// near-threshold columns of each instance (|kq_m| < thr, the first `cap` in index order):
// sel [n_e][cap + 1] int32 = count, indices
ms_status launch_thresh_select(ms_ctx ctx, int n, int n_e, const double2* kq, int64_t sk, double thr, int cap,
                               int32_t* sel);
// A = rho^T (n x n per energy, complex64 when fp32) for the interface product, the columns in sel
// (may be null) left out
ms_status launch_prologue(ms_ctx ctx, int n, int n_e, const double2* Y, int64_t ldy, int64_t sY, const double2* kq,
                          const double2* pq, int64_t sk, const int32_t* sel, int cap, void* Aop, bool fp32);
// M = [Phi_A^T | Phi_B^T] from O, the product W = rho^T [C- | C+ off its diagonal] (null: rho = 0),
// Y, and the FP64 terms of the columns in sel (may be null)
ms_status launch_epilogue(ms_ctx ctx, int n, int n_e, const double2* O, const double2* Wg, const double2* kp,
                          const double2* kq, const double2* pq, int64_t sk, const double2* Y, int64_t ldy, int64_t sY,
                          const int32_t* sel, int cap, double2* M, int64_t ldm, int64_t sM);
ms_status launch_tcols(ms_ctx ctx, int n, int n_o, int n_e, const int32_t* ch, const double2* Y, int64_t ldy,
                       int64_t sY, int y_off, const double2* kq, const double2* pq, int64_t sk, int first, double2* M,
                       int64_t ldm, int64_t sM);
ms_status launch_batch_T(ms_ctx ctx, int n, int n_o, int n_e, const int32_t* ch, const double* energies,
                         const double* eps_l, const double* eps_r, const double2* Y, int64_t ldy, int64_t sY, double* T,
                         double* R, int64_t* n_open, int32_t* status);
ms_status launch_whole_T(ms_ctx ctx, int n, double E, const double2* t, const double2* r, const double* eps_l,
                         const double* eps_r, double* T, double* R, int64_t* n_open, int32_t* status);
ms_status launch_xy(ms_ctx ctx, int n, int nb, const double2* ovl, const double2* kbuf, int p0, double2* aug,
                    double2* Xc, double2* Yc);
ms_status launch_smat_finish(ms_ctx ctx, int n, int nb, const double2* Z, const double2* Xc, const double2* pbuf,
                             int p0, double2* tout, double2* rpout, double2* tpout);
ms_status launch_star_aug(ms_ctx ctx, int n, const double2* ta, const double2* rpa, double2* aug);
ms_status launch_to_c64(ms_ctx ctx, int64_t count, const double2* in, float2* out);
ms_status launch_kpar_average(ms_ctx ctx, int64_t n_k, int64_t n_e, const double* T, const int64_t* n_open,
                               double* tbar, double* per_channel);
ms_status launch_nonfinite_scan(ms_ctx ctx, int64_t count, const double2* v, int32_t* status);
// mixed doubling (App. A, Eq. recurrence2)
ms_status launch_transfer_blocks(ms_ctx ctx, int n, int nb, const double2* ovl, const double2* kbuf,
                                 const double2* pbuf, int p0, double2* I11, double2* I12);
ms_status launch_aug_build(ms_ctx ctx, int n, int nb, int w, const double2* src, int64_t s_src, const double2* src2,
                           int64_t s_src2, const double2* src3, int64_t s_src3, double2* aug);
ms_status launch_axpby(ms_ctx ctx, int64_t nn, int nb, double alpha, const double2* a, int64_t s_a, double beta,
                       const double2* c, int64_t s_c, double2* out, int64_t s_o);
ms_status launch_norm1(ms_ctx ctx, int n, int nb, const double2* A, int64_t ld, int64_t s, double* out);

// first variation of T with respect to the slice potentials (batched over energies: every
// pointer of batch entry b is advanced by b times its stride)
ms_status launch_grad_open_system(ms_ctx ctx, int n, int nl, int nr, const int32_t* olt, const int32_t* ort,
                                  const double2* r, const double2* tpc, const double2* trow, const double2* rpo,
                                  int64_t s_st, double2* aug, int batch);
ms_status launch_gather2(ms_ctx ctx, int nrow, int ncol, const int32_t* rows, const int32_t* cols,
                         const double2* src, int64_t lds, double2* dst, int64_t ldd, int batch = 1, int64_t s_rows = 0,
                         int64_t s_cols = 0, int64_t s_src = 0, int64_t s_dst = 0);
ms_status launch_scatter_rows(ms_ctx ctx, int nrow, int n, const int32_t* rows, const double2* src, double2* dst);
ms_status launch_gather_cols(ms_ctx ctx, int n, int nc, const int32_t* idx, const double2* src, int64_t lds,
                             double2* dst, int64_t ldd);
ms_status launch_grad_p(ms_ctx ctx, int n, int nl, int nr, const double2* c, int64_t ldc, int64_t s_c,
                        const double2* d, int64_t ldd, int64_t s_d, const double2* trow, int64_t s_trow,
                        const int32_t* ol, int64_t s_ol, const double2* kl, int64_t s_kl, double2* p1, double2* p2,
                        int64_t s_p, int batch);
ms_status launch_grad_m(ms_ctx ctx, int n, int nl, const double2* k, int64_t s_k, double width, const double2* p1,
                        const double2* p2, int64_t s_p, const double2* a, int64_t lda, int64_t s_a, const double2* b,
                        int64_t ldb, int64_t s_b, double2* mc, int64_t s_m, int batch);
ms_status launch_eye(ms_ctx ctx, int n, int64_t ld, double2* dst, int batch = 1, int64_t s_dst = 0);
// P, Q of an electrode cell's Bloch eigenproblem from its S-matrix blocks
ms_status launch_bloch_pencil(ms_ctx ctx, int n, const double2* t, const double2* rp, const double2* r,
                              const double2* tp, double2* P, double2* Q);
ms_status launch_grad_scatter(ms_ctx ctx, int64_t nn, const int32_t* q, const double2* kc, int64_t s_kc, double* g,
                              int64_t s_g, int batch);

}  // namespace ms
