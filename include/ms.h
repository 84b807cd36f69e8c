/*
 * ms.h -- C ABI of the MI355X plane-wave multiple-scattering transport library.
 *
 * Method: Li, Chu, Zhang, Cheng, "Electron transport in graphene/graphene
 * side-contact junction by plane-wave multiple scattering method"
 * (arXiv:1504.01462).  Local-potential form: -nabla^2 psi + V psi = E psi
 * (Rydberg units, hbar^2/2m = 1, lengths in bohr), V periodic in the
 * transverse plane and z-independent inside each slice, constant in the two
 * leads.  The non-local projector terms (C, H^a, H^b, h^a, h^b) are zero.
 *
 * Conventions shared by every entry point
 *   - Complex numbers are interleaved {re, im}; c128 = two doubles.  Matrices
 *     are row-major and contiguous (leading dimension = number of columns).
 *   - Every array argument is DEVICE memory of the context's device, except
 *     the small host arrays named `bvec`, `kpar` and `energies`.
 *   - The caller allocates and owns every input and output buffer.  The
 *     context owns only its workspace (grown on demand, freed at destroy).
 *   - Calls enqueue work on the context's stream and return at once.
 *     Argument errors are returned synchronously and enqueue nothing.
 *     Numerical problems found on the device (zero pivot, non-finite data)
 *     are recorded in the context's device status word and returned by
 *     ms_ctx_sync; ms_transmission_batch also writes one status per point.
 *   - Output values are unspecified for points whose status is not MS_OK.
 *   - A context is used by one host thread at a time.
 *
 * Notation (paper, Sec. II.A and App. A): slices p = 1..N between the left
 * lead (p = 0) and the right lead (p = N+1); slice p ends at its reference
 * plane z_p; its modes are the eigenpairs (E^p_n, U^p[:,n]) of the
 * transverse Hamiltonian (Eq. loc); k^p_n = sqrt(E - E^p_n) with Im k >= 0.
 * S(p,p+1) maps [A^p; B^{p+1}] to [A^{p+1}; B^p] (Eq. smm2); its blocks
 * S11, S12, S21, S22 are called t, rp, r, tp here.
 */
#ifndef MS_H
#define MS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MS_OK = 0,
  MS_ERR_ARG = 1,          /* bad size, null pointer, inconsistent arguments            */
  MS_ERR_ALLOC = 2,        /* device workspace allocation failed                         */
  MS_ERR_HIP = 3,          /* a HIP runtime call failed                                  */
  MS_ERR_SINGULAR = 4,     /* exact zero pivot in an LU factorisation (X, I - S12 S21,   */
                           /* or the fused interface matrix)                             */
  MS_ERR_THRESHOLD = 5,    /* |E - lead channel energy| < 1e-10: k = 0 in a lead          */
  MS_ERR_NONFINITE = 6,    /* NaN or Inf met in inputs or results                        */
  MS_ERR_UNSUPPORTED = 7,  /* size or mode the library does not handle                 */
  MS_ERR_NOCONV = 8        /* slice eigensolver did not reach its tolerance              */
} ms_status;

typedef enum {
  MS_PREC_FP64 = 0,        /* every step in FP64 (complex128)                            */
  MS_PREC_FP32_MFMA = 1    /* star-product GEMMs on FP32 MFMA (complex64 operands, FP32  */
                           /* accumulation within each 16-deep K-slab, slabs summed in  */
                           /* FP64); factorisation, solves, the exactly known diagonal  */
                           /* and near-threshold terms and all scalings in FP64         */
} ms_prec;

typedef struct ms_ctx_s* ms_ctx;

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  Fails with MS_ERR_HIP
 * when the device cannot be selected. */
ms_status ms_ctx_create(int device, void* hip_stream, ms_ctx* out);

/* Wait for the context's stream, free its workspace and the context. */
ms_status ms_ctx_destroy(ms_ctx ctx);

/* Wait for all work on the context's stream; return the first numerical
 * status recorded on the device since the last sync (then clear it). */
ms_status ms_ctx_sync(ms_ctx ctx);

/* Static, NUL-terminated name of a status code. */
const char* ms_status_str(ms_status s);

/* Copy the last error message of `ctx` (or of the most recent failed
 * ms_ctx_create when ctx is NULL) into buf (NUL-terminated, at most len). */
ms_status ms_ctx_last_error(ms_ctx ctx, char* buf, int64_t len);

/* One scattering matrix: four n x n c128 blocks in device memory.
 * t = S11, rp = S12, r = S21, tp = S22 (Eq. smm2 and Eq. scatter). */
typedef struct {
  int64_t n;
  void* t;
  void* rp;
  void* r;
  void* tp;
} ms_smat;

/* E-independent slice data of one k_par (filled by ms_slices_prepare).
 *   dz   [n_slices]                 slice thicknesses (bohr); slice p+1 is dz[p]
 *   eps  [n_slices+2][n_g] f64      E^p_n ascending; row 0 = left lead,
 *                                   row n_slices+1 = right lead (|k+G|^2 + V_lead)
 *   ovl  [n_slices+1][n_g][n_g] c128  O^p = U^p^dagger U^{p+1}, p = 0..n_slices
 *                                   (the overlap sum of App. A, Eq. app), with
 *                                   U^0 = U^{n_slices+1} = I
 *   evec [n_slices][n_g][n_g] c128  optional (may be NULL): U^p of slice p+1 as
 *                                   columns (unit norm), matching eps rows 1..n_slices */
typedef struct {
  int64_t n_g;
  int64_t n_slices;
  const double* dz;
  double* eps;
  void* ovl;
  void* evec;
} ms_slices;

/* a1-a3: slice Hamiltonians, their eigenpairs and the interface overlaps.
 *   H^p_ij = |k_par + G_i|^2 delta_ij + V^p(G_i - G_j)        (Sec. II.A, Eq. loc)
 * with G_i = g_mn[i][0] b1 + g_mn[i][1] b2.
 *   g_mn     [n_g][2] int32 (device)  Miller indices of the basis
 *   bvec     [4] f64 (host)           b1x, b1y, b2x, b2y (bohr^-1)
 *   kpar     [2] f64 (host)           k_par (bohr^-1)
 *   vlead_left, vlead_right           constant lead potentials (Ry)
 *   q_of_ij  [n_g][n_g] int32 (device) index into vq's second axis of G_i - G_j
 *   vq       [n_slices][n_q] c128 (device)  V^p(Q); must be Hermitian:
 *            vq[p][q_of_ij[j][i]] = conj(vq[p][q_of_ij[i][j]])
 *   inout    n_g, n_slices, dz, eps, ovl set by the caller (evec optional)
 * Errors: MS_ERR_ARG (sizes, nulls), MS_ERR_UNSUPPORTED (n_g > 4096),
 * MS_ERR_NOCONV / MS_ERR_NONFINITE via ms_ctx_sync. */
ms_status ms_slices_prepare(ms_ctx ctx, int64_t n_g, const int32_t* g_mn, const double* bvec,
                            const double* kpar, double vlead_left, double vlead_right,
                            int64_t n_slices, int64_t n_q, const int32_t* q_of_ij,
                            const void* vq, ms_slices* inout);

/* a4: S(p,p+1) for p = p0 .. p1-1 at energy E (App. A, Eqs. app, bpp,
 * transfer and scatter), in the form with the growing factor cancelled:
 *   X_nj = O_nj (k^p_n + k^{p+1}_j) / (2 k^p_n),  Y_nj = O_nj (k^p_n - k^{p+1}_j) / (2 k^p_n),
 *   P = diag exp(i k^{p+1} dz_{p+1})  (dz of the right lead = 0),
 *   S11 = P X^-1,  S12 = -P X^-1 Y P,  S21 = Y X^-1,  S22 = (X - Y X^-1 Y) P.
 * out[i] receives S(p0+i, p0+i+1); out[i].n must equal slices->n_g.
 * Errors: MS_ERR_ARG; MS_ERR_SINGULAR via ms_ctx_sync when X has a zero pivot. */
ms_status ms_slice_smatrix(ms_ctx ctx, const ms_slices* slices, double energy, int64_t p0,
                           int64_t p1, const ms_smat* out);

/* a5: whole = s[0] * s[1] * ... * s[n-1], the star (layer-doubling) product of
 * Sec. II.A, Eq. recurrence1 (App. A, Eq. recurrence) for a = S(m,n), b = S(n,k):
 *   F = I - S12(a) S21(b)
 *   S11 = S11(b) F^-1 S11(a)             S12 = S12(b) + S11(b) F^-1 S12(a) S22(b)
 *   S21 = S21(a) + S22(a) S21(b) F^-1 S11(a)
 *   S22 = S22(a) S22(b) + S22(a) S21(b) F^-1 S12(a) S22(b)
 * The inputs are not modified; `whole` must not alias them.  The blocks are c128 in both
 * forms.  prec = MS_PREC_FP64: every step in FP64.  prec = MS_PREC_FP32_MFMA: F = I - S12(a)
 * S21(b), its LU factorisation and the solves with it stay FP64; the six products that
 * follow (S22(a) S21(b), S11(b) W1, ..., their sums) run on FP32 MFMA, their operands rounded
 * to c64 (FP32 accumulation within 16-deep K-slabs, slabs summed in FP64).
 * Errors: MS_ERR_ARG (sizes, nulls, aliasing, unknown prec); MS_ERR_SINGULAR via ms_ctx_sync
 * when F has a zero pivot. */
ms_status ms_star_cascade(ms_ctx ctx, const ms_smat* s, int64_t n, ms_prec prec, ms_smat* whole);

/* a6: T, R and the open-channel count of the whole junction for waves
 * incident from the left (App. C: A^0 = I, B^{N+1} = 0, so t = S11 and
 * r = S21), flux-normalised over the open channels O = {n : eps_n < E}:
 *   T = sum_{i in O_right, j in O_left} (k_i / k_j) |t_ij|^2,
 *   R = sum_{i, j in O_left} (k_i / k_j) |r_ij|^2.
 *   eps_left, eps_right [n] f64 (device)  lead channel energies
 *   T, R [1] f64, n_open [1] int64 (device outputs)
 * Errors: MS_ERR_ARG; MS_ERR_THRESHOLD via ms_ctx_sync. */
ms_status ms_transmission(ms_ctx ctx, const ms_smat* whole, double energy, const double* eps_left,
                          const double* eps_right, double* T, double* R, int64_t* n_open);

/* The doubling of App. A with the mixed recurrence (after Eq. recurrence2): the
 * interface blocks (I11, I12, S21, S22) of every S(p,p+1), p = 0..n_slices, with
 *   I11 = X P^-1, I12 = Y P  (Eq. transfer),  S21, S22 as in ms_slice_smatrix,
 * are combined pairwise, level after level (pairs formed left to right; an odd last
 * block moves up unchanged), by
 *   M = I11(m,n) + I12(m,n) S21(n,k),   I11(m,k) = M I11(n,k),
 *   I12(m,k) = M I12(n,k) + I12(m,n) S22(n,k),
 *   S21(m,k) = S21(m,n) + S22(m,n) S21(n,k) M^-1,
 *   S22(m,k) = S22(m,n) S22(n,k) - S22(m,n) S21(n,k) M^-1 I12(m,n) S22(n,k),
 * while the 1-norm condition number ||I11||_1 ||I11^-1||_1 of every block stays at
 * or below max_cond; then every block becomes S by Eq. scatter (S11 = I11^-1,
 * S12 = -I11^-1 I12) and the remaining levels use the star product (Eq. recurrence).
 *   max_cond      >= 1; +inf keeps the mixed form to the end, 1 uses S throughout
 *   whole         the S-matrix of the whole junction (four distinct n_g x n_g blocks)
 *   mixed_levels  [1] int32 (host): number of levels done in the mixed form
 * The condition numbers are read back after every mixed level (the call waits for
 * the stream then).  Workspace: about (6 + 4.5) (n_slices + 1) n_g^2 c128.
 * Errors: MS_ERR_ARG, MS_ERR_ALLOC; MS_ERR_SINGULAR via ms_ctx_sync. */
ms_status ms_mixed_doubling(ms_ctx ctx, const ms_slices* slices, double energy, double max_cond, ms_smat* whole,
                            int32_t* mixed_levels);

/* a4+a5+a6 fused, batched over energies that share the slice data (Sec. II.A, Eqs. smm2 and
 * recurrence1; App. A, Eqs. transfer, scatter and recurrence; App. C with A^0 = I,
 * B^{N+1} = 0): the interfaces are folded from the right lead to the left one; each step is
 * the star product of S(p,p+1) with the accumulated right part, written so that one LU
 * factorisation per interface and energy serves both the slice matrix X and
 * F = I - S12 S21 (exactly equal up to rounding).  No S(p,p+1) is stored.  With
 * rho = P r P the accumulated reflection at slice p+1 and C+- = O^T K_p +- K_{p+1} O^T:
 *   Phi_A^T = C+ + rho^T C-,   Phi_B^T = C- + rho^T C+,   r_new^T = K_p (Phi_A^-T Phi_B^T) K_p^-1
 * (the transmitted columns ride along as right-hand sides).  The products rho^T C+- are the
 * interface GEMM; prec = MS_PREC_FP32_MFMA runs it on FP32 MFMA, with the diagonal of C+ and
 * the columns of rho^T whose |k_{p+1}| < 0.1 (at most 8 per interface, near a slice
 * threshold, where rho grows like |k|^-1/2) added in FP64.
 *   energies   [n_e] f64 (host)
 *   T, R       [n_e] f64 (device outputs)
 *   n_open     [n_e] int64 (device output)
 *   point_status [n_e] int32 (device output; ms_status per point)
 * Errors: MS_ERR_ARG, MS_ERR_UNSUPPORTED (n_g > 4096), MS_ERR_ALLOC. */
ms_status ms_transmission_batch(ms_ctx ctx, const ms_slices* slices, int64_t n_e,
                                const double* energies, ms_prec prec, double* T, double* R,
                                int64_t* n_open, int32_t* point_status);

/* ms_transmission_batch for n_k slice sets at once (several k_par of one junction; the
 * k_par mesh of Sec. II.B, Eq. T1_d), n_e energies each: slices [n_k] (equal n_g and
 * n_slices), energies [n_k][n_e] (host), T, R [n_k][n_e] f64, n_open [n_k][n_e] int64,
 * point_status [n_k][n_e] int32 (device).  The LU factorisations and back substitutions of all
 * n_k * n_e points run as one batch per interface, which amortises their latency-bound panel
 * steps over more matrices.
 * Errors: MS_ERR_ARG (sizes differ between sets, nulls, non-finite energies),
 * MS_ERR_UNSUPPORTED (n_k > 65535), MS_ERR_ALLOC. */
ms_status ms_transmission_multi(ms_ctx ctx, int64_t n_k, const ms_slices* slices, int64_t n_e,
                                const double* energies, ms_prec prec, double* T, double* R, int64_t* n_open,
                                int32_t* point_status);

/* ms_transmission_batch for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same fold, kernels and
 * results, with every scratch buffer carved from one array of MS_NOALLOC_SCRATCH_MAX bytes
 * that the library holds on each device it runs on (a static device array, present until the
 * process ends).  It calls no hipMalloc, hipFree or allocating library routine, creates no
 * stream or event (so no look-ahead LU and no event profiling), and grows no context
 * workspace.  The energies are folded in as many sub-batches as the scratch requires; one
 * instance (one energy of the set) needs about (2 (n_slices + 2) + 5 n_g + n_open) n_g c128
 * plus the LU's workspace, so n_g = 300 takes about 10 per sub-batch, n_g = 1200 none.
 * Every call on a device uses the same array and leaves its contents behind; the call sets
 * what must start at zero itself.  Calls on one device that overlap in time (several
 * contexts or streams, several host threads) race on the array: keep them ordered.
 * Arguments, outputs, status per point and the other errors as ms_transmission_batch;
 * MS_ERR_UNSUPPORTED (nothing enqueued) when one instance or the call's tables do not fit. */
#define MS_NOALLOC_SCRATCH_MAX (128LL << 20)
ms_status ms_transmission_batch_noalloc(ms_ctx ctx, const ms_slices* slices, int64_t n_e,
                                        const double* energies, ms_prec prec, double* T, double* R,
                                        int64_t* n_open, int32_t* point_status);

/* Flag of ms_transmission_uneven: capture the whole fold into one hipGraph and launch it. */
#define MS_FOLD_GRAPH 1

/* The fused fold for slice sets of uneven sizes (n_g and n_slices may differ from set to
 * set), each with its own energies: many independent (E, k_par) instances in one call.
 * Sets of equal n_g form one batch whose LU factorisations and back substitutions run
 * together per fold step; inside it the sets are folded longest first and a set leaves
 * the batch once its left lead is reached (the T of each point is that of
 * ms_transmission_batch for its set and energy, up to rounding).
 *   sets        [n_sets] slice sets (device data, as for ms_transmission_batch)
 *   n_e         [n_sets] int64 (host): energies of each set (0 allowed)
 *   energies    [sum n_e] f64 (host), set 0's first, then set 1's, ...
 *   flags       0 or MS_FOLD_GRAPH: all kernels of the call are captured (on an internal
 *               stream) into one hipGraph, launched once on the context's stream and kept
 *               by the context for ms_graph_replay (until the next capture or destroy);
 *               the graph has a workspace of its own, which other calls do not touch.
 *               One graph holds at most 96000 kernels (about 300 per fold step at
 *               n_g = 1200, 200 at 800, 115 at 450, 55 at 200, times the longest set's
 *               n_slices per n_g group); a larger fold fails with MS_ERR_UNSUPPORTED
 *               (nothing launched) and is run by several calls or without the flag
 *   T, R        [sum n_e] f64, n_open [sum n_e] int64, point_status [sum n_e] int32
 *               (device outputs, in the order of `energies`)
 * Before launching, the call reads each set's right-lead channel energies (it waits for
 * the stream then) and grows its workspace; nothing is allocated inside a capture.
 * Errors: MS_ERR_ARG (nulls, negative counts, unknown flags or precision, non-finite
 * energies), MS_ERR_UNSUPPORTED (n_g > 4096, graph too large), MS_ERR_ALLOC,
 * MS_ERR_HIP (capture). */
ms_status ms_transmission_uneven(ms_ctx ctx, int64_t n_sets, const ms_slices* sets, const int64_t* n_e,
                                 const double* energies, ms_prec prec, int32_t flags, double* T, double* R,
                                 int64_t* n_open, int32_t* point_status);

/* Gradient of T(E) with respect to every Fourier coefficient of every slice potential (the
 * sliced model of Sec. II: H^p_ab = |k+G_a|^2 delta_ab + V^p(G_a - G_b), Eq. loc), from the
 * first variation dt_ij = (1/(2 i k_i)) int phi_i^dagger dH psi_j dz of the transmission
 * amplitudes: psi_j enters from the left in open channel j, phi_i leaves only into the right
 * lead's open channel i; their amplitudes in slice p come from the star-product cascades
 * S(0,p) and S(p,N+1) (Sec. II.A, Eqs. smm2 and recurrence1).  Output g with
 *   dT = 2 Re sum_{p,Q} g[p][Q] dV^p(Q)
 * to first order, for independent complex dV (keep V(-Q) = conj V(Q) to stay Hermitian:
 * dT/dRe V(Q) = 2 Re(g(Q) + g(-Q)), dT/dIm V(Q) = 2 Im(g(-Q) - g(Q)) for Q != -Q).
 *   slices      prepared with the eigenvectors (slices->evec != NULL)
 *   energies    [n_e] f64 (host); the energies go through every launch together, in
 *               batches of at most 16 and of as many as 3/4 of the free device memory holds
 *   q_of_ij     [n_g][n_g] int32 (device), the map of ms_slices_prepare
 *   n_q         number of Q
 *   checkpoint  planes between stored right cascades; those between are recomputed segment
 *               by segment (1: every plane kept, none recomputed; 0: 1 when that fits the
 *               energies in flight into 3/4 of the free device memory, else about
 *               sqrt(n_slices + 1)); workspace per energy of a batch about 4 (L + 1) +
 *               (n_slices + 1) / checkpoint + checkpoint + 12 blocks of n_g^2 c128, L =
 *               checkpoint (16 when checkpoint is 1)
 *   grad        [n_e][n_slices][n_q] c128 (device output)
 *   t_r         [n_e][2] f64 (device output): T and R; n_open [n_e] int64 (device)
 * The cascades carry only what the amplitudes need (S(p,N+1): r, the open columns of t', the
 * open rows of t, the open block of r'; S(0,p): r', the open columns of t).  Cost per
 * interface and energy: two such star products (4 1/3 n_g^3 complex MACs each), a third to
 * recompute the right cascade where it is not stored, two slice S-matrices (4 n_g^3 each)
 * and, per slice, I - L12 R21, its LU and conj(U) M U^T (3 1/3 n_g^3): about 20 n_g^3 with
 * every plane kept, about 24 1/3 n_g^3 otherwise.
 * The sum over Q uses FP64 atomic additions, so g can differ in the last bits from run to
 * run (T and R do not).  Waits for the stream (the range of q_of_ij, the lead channel
 * energies, each slice S-matrix segment).
 * Errors: MS_ERR_ARG (no eigenvectors, nulls, non-finite energies, n_q < 1, q_of_ij out of
 * [0, n_q)), MS_ERR_UNSUPPORTED, MS_ERR_ALLOC; numerical errors (singular systems, lead
 * threshold) via ms_ctx_sync. */
ms_status ms_dT_dV(ms_ctx ctx, const ms_slices* slices, int64_t n_e, const double* energies, const int32_t* q_of_ij,
                   int64_t n_q, int64_t checkpoint, void* grad, double* t_r, int64_t* n_open);

/* Tile edges of the fold's complex GEMMs for one basis size: 64 (64 x 64 tiles, 4 waves) or
 * 128 (128 x 64 tiles, 8 waves; FP64 products only, the FP32-MFMA form always takes 64); 0 =
 * the default (64).  Roles: the interface product (Sec. II, the
 * star product with the accumulated right part), the LU's rank-128 trailing update, and its
 * in-panel and U12 products.  Both shapes accumulate every element in the same order, so the
 * edges change run time only, never a result. */
typedef struct {
  int32_t iface, lu_update, lu_inner;
} ms_tiles;

/* Use `tiles` for every fold group of basis size n_g on this context.
 * Errors: MS_ERR_ARG (n_g < 1, an edge other than 0, 64, 128, NULL). */
ms_status ms_set_tiles(ms_ctx ctx, int64_t n_g, const ms_tiles* tiles);

/* Autotuner: for basis size n_g, n_open open channels and `batch` systems per fold step
 * (at most 64 are used), time on the device the LU factorisation + back substitution of
 * synthetic augmented systems (n_g x (2 n_g + n_open), dominant diagonal) with each pair of
 * (trailing-update, in-panel) edges and the stacked interface product with each edge, best
 * of two runs each; record the fastest per role for n_g (as ms_set_tiles) and return them in
 * `chosen`.  times_ms (optional, host [6]): LU 64/64, 64/128, 128/64, 128/128, interface 64,
 * interface 128.  Waits for the stream.  Workspace: about batch (5 n_g^2 + n_g n_open) c128.
 * Errors: MS_ERR_ARG, MS_ERR_UNSUPPORTED (inside a capture), MS_ERR_ALLOC, MS_ERR_HIP. */
ms_status ms_autotune(ms_ctx ctx, int64_t n_g, int64_t n_open, int64_t batch, ms_tiles* chosen, double* times_ms);

/* Launch the graph captured by the last ms_transmission_uneven(..., MS_FOLD_GRAPH, ...) on
 * this context again, on the context's stream.  The graph reads the slice sets' device data
 * (eps, ovl, dz) and writes the output buffers given at capture, whose contents may have
 * changed since (e.g. the same Slices buffers prepared again from another potential); their
 * sizes and addresses may not.  Fixed at capture are the energies and each set's right-lead
 * open-channel table (read from eps at the set's highest energy): a replay after changing the
 * lead channel energies (another k_par or lead potential) folds with the captured channel
 * columns, so capture again then.
 * Errors: MS_ERR_ARG (no graph), MS_ERR_HIP. */
ms_status ms_graph_replay(ms_ctx ctx);

/* a7: average over the k_par mesh (Sec. II.B, Eq. T1_d):
 *   tbar[e]        = (1/n_k) sum_k T[k][e]
 *   per_channel[e] = sum_k T[k][e] / sum_k n_open[k][e]   (0 when no channel is open)
 *   T [n_k][n_e] f64, n_open [n_k][n_e] int64, tbar, per_channel [n_e] f64 (device).
 * Errors: MS_ERR_ARG. */
ms_status ms_kpar_average(ms_ctx ctx, int64_t n_k, int64_t n_e, const double* T, const int64_t* n_open,
                          double* tbar, double* per_channel);

/* Electrode cell, first stage of the complex bands (App. B, Eq. cmp; local potential, so no
 * non-local sphere crosses a cell boundary): the Bloch conditions A^{M+1} = lam A^1,
 * B^{M+1} = lam B^1 (lam = e^{ikd}) through the cell's S-matrix S = S(1, M+1), with the cell's
 * incoming amplitudes X = [A^1; B^{M+1}] as unknowns, give P X = lam Q X with
 *   P = [[S11, S12], [0, I]],  Q = [[I, 0], [S21, S22]]   (2 n_g x 2 n_g).
 *   cell    the cell's slices 1..M (n_slices = M >= 1), prepared by ms_slices_prepare WITH
 *           the eigenvectors (cell->evec); the lead entries are unused.  Slice M+1 is the next
 *           cell's slice 1: the last interface S(M, M+1) uses O = U^M^dagger U^1 of the cell's
 *           own eigenvectors, dz_1 and slice 1's channel energies, so both Bloch planes are
 *           reference planes of one and the same slice-1 eigenbasis
 *   P, Q    [2 n_g][2 n_g] c128 (device outputs, row-major, distinct)
 * The pencil's eigenvalues lam and eigenvectors (A^1 and B^{M+1} both in slice 1's
 * eigenbasis) are the electrode's Bloch states; solving it is not part of the library yet.
 * Errors: MS_ERR_ARG (no eigenvectors, nulls, non-finite energy), MS_ERR_UNSUPPORTED,
 * MS_ERR_ALLOC; singular X or F via ms_ctx_sync. */
ms_status ms_bloch_pencil(ms_ctx ctx, const ms_slices* cell, double energy, void* P, void* Q);

/* Complex band structure of an electrode cell at one energy (App. B, Eq. cmp): the 2 n_g Bloch
 * states of the pencil P X = lam Q X of ms_bloch_pencil, by a complex QZ iteration (unitary
 * reduction of (P, Q) to upper triangular (S, T), one workgroup per pencil): lam_k = alpha_k /
 * beta_k, kept as pairs so that states changing by more than FP64 spans over one cell stay exact
 * (beta_k = 0: an infinite lam), and the right eigenvectors [A^1; B^{M+1}] in the cell's slice-1
 * eigenbasis.
 *   cell     the cell's slices 1..M prepared with eigenvectors (as for ms_bloch_pencil)
 *   alpha, beta [2 n_g] c128 (device outputs; beta real >= 0)
 *   X        [2 n_g][2 n_g] c128 (device output; column k = state k, unit 2-norm)
 * Waits for the stream (the iteration's convergence status).  Errors: MS_ERR_ARG,
 * MS_ERR_UNSUPPORTED (n_g > 2048), MS_ERR_NOCONV (more than 30 sweeps per eigenvalue), MS_ERR_ALLOC. */
ms_status ms_complex_bands(ms_ctx ctx, const ms_slices* cell, double energy, void* alpha, void* beta, void* X);

/* Transmission between two periodic electrodes through a scattering region (App. C, Eq. trans,
 * in the S-matrix form of Sec. II.A; the electrodes' Bloch states of App. B, Eq. cmp).  The left
 * electrode ends with a copy of its cell's slice 1, the region's slices follow, the right
 * electrode starts with its cell's slice 1; S = S(L1, R1) joins those two reference planes.
 * Each electrode's 2 n_g Bloch states (ms_complex_bands) are read at the slice-1 plane where each
 * is largest (|lam| <= 1: (A^1, S21 A^1 + S22 B^{M+1}); otherwise (S11 A^1 + S12 B^{M+1},
 * B^{M+1}), no division by lam) and sorted by direction: propagating (||lam| - 1| < 1e-8) by the
 * sign of their flux, evanescent by |lam| (decaying towards +z: right-going).  Per incident
 * (right-going propagating) state of the left electrode, the 2 n_g amplitudes tau of the right
 * electrode's right-going states and rho of the left electrode's left-going states solve
 *   T_a tau = S11 (a_in + R_a rho) + S12 T_b tau,   b_in + R_b rho = S21 (a_in + R_a rho) + S22 T_b tau,
 * and with the states' flux matrices J(u, v) = (a_u + b_u)^H K (a_v - b_v) + (a_u - b_u)^H K^* (a_v + b_v):
 *   T = Re Tr[(tau_p^H J_out tau_p) J_in^-1],  R = Re Tr[(rho_p^H J_ref rho_p) J_in^-1]
 * over the propagating transmitted and reflected states (valid for degenerate states too).
 *   left, right   electrode cells (slices 1..M, eigenvectors kept); region: the scattering
 *                 region's slices, eigenvectors kept; one n_g for all three (same basis)
 *   T, R [1] f64, n_in [1] int64 (device outputs): n_in incident states, T + R = n_in
 * Waits for the stream.  Errors: MS_ERR_ARG, MS_ERR_UNSUPPORTED (n_g > 2048, more than 24
 * propagating states per direction), MS_ERR_THRESHOLD (not n_g states per direction: an energy
 * at a band edge), MS_ERR_NOCONV; a singular matching system via ms_ctx_sync. */
ms_status ms_electrode_transmission(ms_ctx ctx, const ms_slices* left, const ms_slices* region,
                                    const ms_slices* right, double energy, double* T, double* R, int64_t* n_in);

/* ms_electrode_transmission at n_e energies (host array energies [n_e], 1 <= n_e <= 32768):
 * T, R [n_e] f64 and n_in [n_e] int64 device outputs.  Both electrodes' pencils at every energy
 * are solved in one QZ launch (one workgroup per pencil, 2 n_e pencils; in chunks of at most
 * 48 GiB of pencil buffers), then each energy is matched as in the single call, whose results
 * it reproduces bit for bit.  Waits for the stream.  Errors: as ms_electrode_transmission; the
 * first energy that fails names its index in the error text. */
ms_status ms_electrode_transmission_batch(ms_ctx ctx, const ms_slices* left, const ms_slices* region,
                                          const ms_slices* right, int64_t n_e, const double* energies, double* T,
                                          double* R, int64_t* n_in);

#ifdef __cplusplus
}
#endif

#endif /* MS_H */
