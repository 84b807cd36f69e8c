// Internal declarations of the MI355X multiple-scattering library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/ms.h"

namespace ms {
// kernel categories timed by the optional event profiler
enum ProfCat {
  PC_IFACE_GEMM = 0,  // the interface GEMM of the fused fold (rho^T O^T, both halves)
  PC_LU_PANEL,        // LU panel factorisation
  PC_LU_SWAP,         // row interchanges + unit-lower solve of the panel rows
  PC_LU_UPDATE,       // rank-128 trailing GEMM update of the LU (right of an outer panel)
  PC_TRSM,            // back substitution
  PC_JACOBI,          // one round of the block Jacobi eigensolver
  PC_PREP_GEMM,       // overlap GEMMs of the E-independent stage
  PC_ELEM,            // elementwise kernels of the fused fold (prologue/epilogue/T)
  PC_OTHER,
  PC_LU_INNER,        // GEMM updates inside an outer panel and the U12 product
  PC_COUNT
};
struct ProfRec {
  hipEvent_t a, b;
  double flops, bytes;
};
}  // namespace ms

struct ms_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t* d_status = nullptr;   // device status word (first error wins)
  std::vector<void*> ws;         // workspace slots, grown on demand
  std::vector<size_t> ws_size;
  std::string last_error;
  uint32_t prof_mask = 0;        // categories timed by the event profiler
  std::vector<ms::ProfRec> prof[ms::PC_COUNT];
  std::vector<hipEvent_t> ev_pool;
  bool owns_status = true;
  std::vector<ms_ctx_s*> kids;   // internal contexts with their own stream and workspace
  std::vector<hipEvent_t> sync_ev;  // fork/join events (reused; destroyed with the context)
  std::vector<hipEvent_t> lu_ev;    // look-ahead events of the LU (reused)
  int jacobi_n = -1;                // n of the round-robin schedule held in workspace slot 10
  void* jacobi_pairs = nullptr;
  bool capturing = false;           // launches go into a hipGraph: no allocation, sync or timing
  hipStream_t cap_stream = nullptr; // stream the captures are recorded on
  hipGraphExec_t graph = nullptr;   // the last captured fold, replayable
  // GEMM tile edges (64 or 128; 0 = default rule) chosen per basis size for the interface
  // product, the LU's rank-128 update and its in-panel / U12 products, and the basis size of
  // the fold group being enqueued (0 outside a fold)
  struct Tiles { int64_t n; int iface, lu_update, lu_inner; };
  std::vector<Tiles> tiles;
  int64_t tile_n = 0;
  int64_t cap_kernels = 0;          // kernels recorded by the open capture
  int64_t cap_limit = 0;            // most kernels one capture may hold
  // workspace owned by the captured graph (its tables and scratch), so that later calls on
  // the context, which use `ws`, neither overwrite nor free what a replay reads
  std::vector<void*> gws;
  std::vector<size_t> gws_size;
  bool use_gws = false;
  // allocation-free mode: every workspace slot is carved from `arena` (a device array of
  // arena_size bytes the library owns), bump-allocated from its start for each call; no
  // device allocation, no event creation, no look-ahead stream
  char* arena = nullptr;
  size_t arena_size = 0, arena_used = 0;
  std::vector<void*> aws;
  std::vector<size_t> aws_size;
};

namespace ms {

// Records HIP events around the launches in its scope when profiling is on.
// With kernel_events = true the scope holds exactly one launch, which passes
// a and b to hipExtLaunchKernel: the events then carry that kernel's own start
// and end instead of the moments the stream reached them, so time spent waiting
// for compute units held by other streams is not counted.
struct Prof {
  ms_ctx ctx;
  int cat;
  double flops, bytes;
  hipEvent_t a = nullptr, b = nullptr;
  bool ext = false;
  Prof(ms_ctx c, int category, double fl = 0.0, double by = 0.0, bool kernel_events = false);
  ~Prof();
};

enum Op { OP_N = 0, OP_T = 1, OP_C = 2 };

// ---- error plumbing -------------------------------------------------------------------
ms_status fail(ms_ctx ctx, ms_status s, const char* fmt, ...);
ms_status hip_fail(ms_ctx ctx, hipError_t e, const char* what);

#define MS_TRY(expr)                         \
  do {                                       \
    ms_status _s = (expr);                   \
    if (_s != MS_OK) return _s;              \
  } while (0)

#define MS_HIP(ctx, expr)                                   \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return ms::hip_fail(ctx, _e, #expr); \
  } while (0)

// workspace slot `slot` of at least `bytes` (synchronises the stream before growing; in the
// allocation-free mode a new region of the arena instead, or MS_ERR_UNSUPPORTED past its end)
ms_status workspace(ms_ctx ctx, int slot, size_t bytes, void** out);
ms_status check_launch(ms_ctx ctx, const char* what);
// internal child context i of ctx (own stream of default priority, own workspace,
// the parent's status word and profiler mask), created on first use
ms_status child(ms_ctx ctx, int i, ms_ctx* out);

// ---- complex GEMM: C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b] (row-major) -------
struct GemmArgs {
  int M = 0, N = 0, K = 0;
  int opA = OP_N, opB = OP_N;
  const void* A = nullptr;
  int64_t lda = 0, sA = 0;
  const void* B = nullptr;
  int64_t ldb = 0, sB = 0;
  double2* C = nullptr;
  int64_t ldc = 0, sC = 0;
  double2 alpha = {1.0, 0.0};
  double2 beta = {0.0, 0.0};
  int batch = 1;
  int prof = PC_OTHER;   // profiler category of this launch
  // The fold's interface product generates its B operand (N = 2 nh columns) from a shared
  // FP64 overlap O (B = O, opB = OP_T, sB = 0) and the wavevectors of batch entry b at
  // kp + b sk (left slice), kq + b sk (right slice):
  //   B_b[m][j] = O[j][m] (kp[j] - kq[m]),  B_b[m][nh + j] = O[j][m] (kp[j] + kq[m]) (0 at m = j)
  const double2* kp = nullptr;
  const double2* kq = nullptr;
  int64_t sk = 0;
  // Optional epilogue of the interface product (ey != nullptr): instead of W = rho^T [C- | C+],
  // C receives the fold's augmented-matrix columns [Phi_A^T | Phi_B^T]:
  //   C[i][j]      = C+_ij + W-_ij + sum_sel rho^T_im O_jm (kp_j - kq_m)
  //   C[i][nh + j] = C-_ij + W+_ij + rho^T_ij C+_jj + sum_sel, m != j rho^T_im O_jm (kp_j + kq_m)
  // with C+-_ij = O_ji (kp_j +- kq_i) and rho^T_im = P_i kq_i Y_im P_m / kq_m from the state Y
  // (ey + b esy, row stride eldy) and the propagators P (epq + b sk); sel (esel + b (ecap + 1):
  // count, then columns) lists the columns rho^T was staged without (null: none)
  const double2* ey = nullptr;
  int64_t eldy = 0, esy = 0;
  const double2* epq = nullptr;
  const int32_t* esel = nullptr;
  int ecap = 0;
};
// A complex128 (B complex128); FP64 MFMA.
ms_status zgemm(ms_ctx ctx, const GemmArgs& g);
// A, B complex64 (a generated B: from the complex128 O, rounded when staged); FP32 MFMA
// with FP32 accumulation; C complex128.
ms_status cgemm32(ms_ctx ctx, const GemmArgs& g);

// ---- batched LU of an augmented matrix and triangular solves (FP64) -------------------
// Factor the leading n x n block of each n x ncols row-major matrix (ld = ncols)
// with partial pivoting; row operations are applied to all ncols columns, so the
// columns [n, ncols) end up holding L^-1 P^T B.  piv: [batch][n] int32.
// status: [batch] int32 (may be null); a zero pivot writes MS_ERR_SINGULAR.
// status index of matrix b is b * sst (sst = 0: one shared word).
ms_status getrf_aug(ms_ctx ctx, double2* A, int n, int ncols, int64_t strideA, int batch,
                    int32_t* piv, int32_t* status, int64_t sst);
// Solve U Y = Z for the upper factor U (leading n x n of A) and Z = A[:, n:ncols];
// Y written to Y (n x (ncols-n), leading dim ldy, batch stride sY).
ms_status trsm_upper_aug(ms_ctx ctx, const double2* A, int n, int ncols, int64_t strideA, int batch,
                         double2* Y, int64_t ldy, int64_t sY, int32_t* status, int64_t sst);

// ---- elementwise and reduction kernels (launchers) ------------------------------------
ms_status launch_kin_eps(ms_ctx ctx, int n, const int32_t* g_mn, const double* bvec, const double* kpar,
                         double vl, double vr, double* kin, double* eps_left, double* eps_right);
// positivity shifts of nb slices whose V(Q) rows are vstride elements apart
ms_status launch_slice_shift(ms_ctx ctx, int n, int nb, const double* kin, int64_t n_q, int64_t vstride,
                             const double2* vq, int q0, double* shift);
// W = H + diag(shift) (shift may be null for H itself); V(Q) rows vstride elements apart
ms_status launch_hgather(ms_ctx ctx, int n, int nb, const double* kin, const double* shift, int64_t vstride,
                         const double2* vq, const int32_t* q_of_ij, double2* W);
// Z[i] = Uref[nearest reference of slice s0 + i] (references every `stride` slices)
ms_status launch_gather_ref(ms_ctx ctx, int n, int nb, int s0, int stride, int nref, const double2* Uref,
                            double2* Z);
// Eigenpairs of nb Hermitian matrices H (n x n each, not modified): W holds (H + c I) V on
// entry for some unitary V (V = I: W = H + c I; a nearby slice's eigenvectors: a warm start),
// and is destroyed; Z is an nb x n x n scratch; eps ascending, U columns = unit eigenvectors.
ms_status jacobi_eigh(ms_ctx ctx, int n, int nb, double2* W, const double2* H, double2* Z, double* eps_out,
                      int64_t eps_stride, double2* U, int64_t u_stride, int32_t* status);
ms_status launch_copy_boundary_overlaps(ms_ctx ctx, int n, const double2* U, double2* O, int conj_transpose);
ms_status launch_minmax(ms_ctx ctx, int64_t count, const int32_t* v, int32_t* out2);
// copy `bytes` of host data to device memory and wait (the host buffer may be temporary)
ms_status upload(ms_ctx ctx, void* dst, const void* src, size_t bytes);

// k and P of rows [0, nrows) for n_e energies; instance e writes kbuf + e * sk (sk <= 0: nrows * n)
ms_status launch_wavevectors(ms_ctx ctx, int n, int nrows, int n_e, const double* eps, const double* energies_dev,
                             const double* dz_rows, double2* kbuf, double2* pbuf, int64_t sk = 0);
ms_status launch_fill_i32(ms_ctx ctx, int64_t count, int32_t* v, int32_t value);
ms_status launch_scatter_results(ms_ctx ctx, int64_t count, const int64_t* perm, const double* t, const double* r,
                                 const int64_t* no, const int32_t* st, double* T, double* R, int64_t* n_open,
                                 int32_t* status);
// workspace of getrf_aug and trsm_upper_aug for `batch` matrices, grown ahead (before a capture)
ms_status lu_reserve(ms_ctx ctx, int n, int ncols, int batch);
// bytes of that workspace per matrix of a batch
size_t lu_bytes_per_matrix(int n, int ncols);

// ---- generalized eigenproblem A x = lam B x (complex QZ, one workgroup per pencil) ---------
// A, B [batch][n][n] are destroyed (S, T); V, Y scratch of the same size; alpha, beta [batch][n]
// (lam = alpha / beta, beta real >= 0); X [batch][n][n] right eigenvectors as unit columns;
// status [batch] (MS_ERR_NOCONV when an eigenvalue needs more than 30 n sweeps in all)
ms_status qz_eig(ms_ctx ctx, int n, int batch, double2* A, double2* B, double2* V, double2* Y, double2* alpha,
                 double2* beta, double2* X, int32_t* status);

}  // namespace ms
