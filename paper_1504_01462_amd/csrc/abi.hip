// C ABI of the MI355X multiple-scattering library: context, workspace, argument
// checking and the orchestration of the kernels (include/ms.h documents the calls).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "elem.h"
#include "ms_internal.h"

static thread_local std::string g_create_error;

// Scratch of the allocation-free entry point (ms_transmission_batch_noalloc): one array per
// device, held by every process that loads the library until it ends.  Host code uses the
// address hipGetSymbolAddress returns for the current device, never the array's name.
constexpr size_t MS_NOALLOC_SCRATCH_BYTES = (size_t)MS_NOALLOC_SCRATCH_MAX;   // include/ms.h
static __device__ __align__(256) unsigned char scratch[MS_NOALLOC_SCRATCH_BYTES];

namespace ms {

ms_status fail(ms_ctx ctx, ms_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->last_error = buf;
  else g_create_error = buf;
  return s;
}

ms_status hip_fail(ms_ctx ctx, hipError_t e, const char* what) {
  const ms_status s = (e == hipErrorOutOfMemory) ? MS_ERR_ALLOC : MS_ERR_HIP;
  return fail(ctx, s, "%s: %s", what, hipGetErrorString(e));
}

ms_status check_launch(ms_ctx ctx, const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, what);
  if (ctx->capturing && ++ctx->cap_kernels > ctx->cap_limit)
    return fail(ctx, MS_ERR_UNSUPPORTED,
                "the fold needs more than %lld kernels in one graph; split the sets over several calls "
                "or call without MS_FOLD_GRAPH", (long long)ctx->cap_limit);
  return MS_OK;
}

ms_status workspace(ms_ctx ctx, int slot, size_t bytes, void** out) {
  if (bytes == 0) bytes = 256;
  if (ctx->arena) {   // allocation-free mode: bump-allocate from the arena
    if ((size_t)slot >= ctx->aws.size()) {
      ctx->aws.resize(slot + 1, nullptr);
      ctx->aws_size.resize(slot + 1, 0);
    }
    if (ctx->aws_size[slot] < bytes) {
      const size_t want = (bytes + 255) & ~(size_t)255;
      if (want > ctx->arena_size - ctx->arena_used)
        return fail(ctx, MS_ERR_UNSUPPORTED,
                    "the call needs more than the %zu bytes of the allocation-free scratch (slot %d, %zu bytes)",
                    ctx->arena_size, slot, bytes);
      ctx->aws[slot] = ctx->arena + ctx->arena_used;
      ctx->aws_size[slot] = want;
      ctx->arena_used += want;
    }
    *out = ctx->aws[slot];
    return MS_OK;
  }
  std::vector<void*>& ws = ctx->use_gws ? ctx->gws : ctx->ws;
  std::vector<size_t>& ws_size = ctx->use_gws ? ctx->gws_size : ctx->ws_size;
  if ((size_t)slot >= ws.size()) {
    ws.resize(slot + 1, nullptr);
    ws_size.resize(slot + 1, 0);
  }
  if (ws_size[slot] < bytes) {
    if (ctx->capturing)   // the planning pass sizes every slot a captured launch uses
      return fail(ctx, MS_ERR_UNSUPPORTED, "workspace slot %d would grow inside a graph capture", slot);
    MS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ws[slot]) MS_HIP(ctx, hipFree(ws[slot]));
    ws[slot] = nullptr;
    ws_size[slot] = 0;
    const size_t want = (bytes + 4095) & ~(size_t)4095;
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) return hip_fail(ctx, e, "workspace hipMalloc");
    ws[slot] = p;
    ws_size[slot] = want;
  }
  *out = ws[slot];
  return MS_OK;
}

static hipEvent_t take_event(ms_ctx ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

Prof::Prof(ms_ctx c, int category, double fl, double by, bool kernel_events)
    : ctx(c), cat(category), flops(fl), bytes(by), ext(kernel_events) {
  if (ctx && !ctx->capturing && !ctx->arena && (ctx->prof_mask >> category & 1u)) {
    a = take_event(ctx);
    if (!a) return;
    if (ext) {
      b = take_event(ctx);
      if (!b) {
        ctx->ev_pool.push_back(a);
        a = nullptr;
      }
    } else {
      (void)hipEventRecord(a, ctx->stream);
    }
  }
}

Prof::~Prof() {
  if (!a) return;
  if (!ext) {
    b = take_event(ctx);
    if (!b) return;
    (void)hipEventRecord(b, ctx->stream);
  }
  ctx->prof[cat].push_back(ProfRec{a, b, flops, bytes});
}

ms_status child(ms_ctx ctx, int i, ms_ctx* out) {
  while ((int)ctx->kids.size() <= i) {
    ms_ctx k = new ms_ctx_s;
    k->device = ctx->device;
    k->d_status = ctx->d_status;
    k->owns_status = false;
    const hipError_t e = hipStreamCreate(&k->stream);
    if (e != hipSuccess) {
      delete k;
      return hip_fail(ctx, e, "hipStreamCreate");
    }
    ctx->kids.push_back(k);
  }
  ctx->kids[i]->prof_mask = ctx->prof_mask;
  *out = ctx->kids[i];
  return MS_OK;
}

ms_status upload(ms_ctx ctx, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return MS_OK;
  MS_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
  MS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return MS_OK;
}

}  // namespace ms

using namespace ms;

namespace {

// workspace slots
enum {
  WS_KIN = 0, WS_SHIFT, WS_W, WS_U, WS_MISC, WS_K, WS_P, WS_AOP, WS_M = 9,
  WS_JPAIRS = 10, WS_JCOUNT = 11,
  WS_Y = 12, WS_PIV, WS_CH, WS_EN, WS_OC, WS_AUG, WS_XC, WS_YC, WS_Z, WS_S4,
  WS_ACC0, WS_ACC1, WS_G, WS_H, WS_V, WS_UREF, WS_PREP_V,
  WS_MD_A = 33, WS_MD_B, WS_MD_INV, WS_MD_T, WS_MD_NRM,
  WS_PERM, WS_RT, WS_RR, WS_RNO, WS_RST,
  // first variation of T
  WS_GSEG, WS_GCK, WS_GRS, WS_GL, WS_GK, WS_GP, WS_GCH, WS_GOS, WS_GX, WS_GFA, WS_GFB, WS_GAUG, WS_GY,
  WS_GT1, WS_GBP, WS_GBF, WS_GP1, WS_GP2, WS_GMC, WS_GYG, WS_GKC, WS_GPIV, WS_GEN, WS_GA2, WS_GB2,
  // electrode cells
  WS_BSEG, WS_BWHOLE, WS_BEPS, WS_BOVL,
  // complex64 operands of the FP32 form of the star product
  WS_S32A, WS_S32B,
  // near-threshold columns of the FP32-MFMA fold
  WS_SEL
};

constexpr int MAX_N = 4096;
constexpr int64_t MAX_GRAPH_KERNELS = 96000;   // kernels one captured fold graph may hold
// bytes of per-energy workspace per sub-batch: 256 instances at N_G = 1200 (108 MB each in
// FP64, 96 MB in FP32) fold in one sub-batch
constexpr size_t BATCH_BUDGET = size_t(32) << 30;
constexpr size_t ARENA_TABLES = size_t(1) << 20;     // arena bytes kept for the fold's tables
// FP32-MFMA fold: columns of rho^T whose |k| in slice p+1 is below THRESH_K (at most THRESH_CAP
// per instance and interface) are taken out of the FP32 product and added in FP64
constexpr double THRESH_K = 0.1;
constexpr int THRESH_CAP = 8;
constexpr size_t PREP_BUDGET = size_t(8) << 30;     // bytes of eigensolver workspace per chunk
constexpr int WARM_STRIDE = 8;                       // reference slices for the warm-started eigensolver

bool bad_ptr(const void* p) { return p == nullptr; }

ms_status check_slices(ms_ctx ctx, const ms_slices* s) {
  if (!s) return fail(ctx, MS_ERR_ARG, "slices is NULL");
  if (s->n_g <= 0 || s->n_slices <= 0) return fail(ctx, MS_ERR_ARG, "n_g and n_slices must be positive");
  if (s->n_g > MAX_N) return fail(ctx, MS_ERR_UNSUPPORTED, "n_g = %lld > %d", (long long)s->n_g, MAX_N);
  if (bad_ptr(s->dz) || bad_ptr(s->eps) || bad_ptr(s->ovl))
    return fail(ctx, MS_ERR_ARG, "slices->dz, eps and ovl must be device pointers");
  return MS_OK;
}

ms_status check_smat(ms_ctx ctx, const ms_smat* s, int64_t n, const char* name) {
  if (!s) return fail(ctx, MS_ERR_ARG, "%s is NULL", name);
  if (s->n != n) return fail(ctx, MS_ERR_ARG, "%s.n = %lld, expected %lld", name, (long long)s->n, (long long)n);
  if (bad_ptr(s->t) || bad_ptr(s->rp) || bad_ptr(s->r) || bad_ptr(s->tp))
    return fail(ctx, MS_ERR_ARG, "%s has a NULL block", name);
  return MS_OK;
}

inline double2* c2(void* p) { return static_cast<double2*>(p); }
inline const double2* c2(const void* p) { return static_cast<const double2*>(p); }

ms_status gemm(ms_ctx ctx, int M, int N, int K, const void* A, int64_t lda, int opA, const void* B, int64_t ldb,
               int opB, void* C, int64_t ldc, double2 alpha, double2 beta) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.opA = opA;
  g.B = B; g.ldb = ldb; g.opB = opB;
  g.C = c2(C); g.ldc = ldc;
  g.alpha = alpha; g.beta = beta;
  return zgemm(ctx, g);
}

const double2 ONE = {1.0, 0.0}, ZERO = {0.0, 0.0}, MONE = {-1.0, 0.0};

}  // namespace

extern "C" {

const char* ms_status_str(ms_status s) {
  switch (s) {
    case MS_OK: return "MS_OK";
    case MS_ERR_ARG: return "MS_ERR_ARG";
    case MS_ERR_ALLOC: return "MS_ERR_ALLOC";
    case MS_ERR_HIP: return "MS_ERR_HIP";
    case MS_ERR_SINGULAR: return "MS_ERR_SINGULAR";
    case MS_ERR_THRESHOLD: return "MS_ERR_THRESHOLD";
    case MS_ERR_NONFINITE: return "MS_ERR_NONFINITE";
    case MS_ERR_UNSUPPORTED: return "MS_ERR_UNSUPPORTED";
    case MS_ERR_NOCONV: return "MS_ERR_NOCONV";
  }
  return "MS_ERR_UNKNOWN";
}

ms_status ms_ctx_last_error(ms_ctx ctx, char* buf, int64_t len) {
  if (!buf || len <= 0) return MS_ERR_ARG;
  const std::string& m = ctx ? ctx->last_error : g_create_error;
  const size_t k = std::min((size_t)(len - 1), m.size());
  memcpy(buf, m.data(), k);
  buf[k] = 0;
  return MS_OK;
}

ms_status ms_ctx_create(int device, void* hip_stream, ms_ctx* out) {
  if (!out) return fail(nullptr, MS_ERR_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0) return fail(nullptr, MS_ERR_HIP, "no HIP device available");
  if (device < 0 || device >= count) return fail(nullptr, MS_ERR_ARG, "device %d out of range [0,%d)", device, count);
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(nullptr, MS_ERR_HIP, "hipSetDevice: %s", hipGetErrorString(e));
  ms_ctx c = new ms_ctx_s;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  e = hipMalloc(&c->d_status, sizeof(int32_t));
  if (e == hipSuccess) e = hipMemsetAsync(c->d_status, 0, sizeof(int32_t), c->stream);
  if (e != hipSuccess) {
    if (c->d_status) (void)hipFree(c->d_status);
    delete c;
    return fail(nullptr, MS_ERR_HIP, "context status word: %s", hipGetErrorString(e));
  }
  *out = c;
  return MS_OK;
}

ms_status ms_ctx_destroy(ms_ctx ctx) {
  if (!ctx) return MS_ERR_ARG;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (ms_ctx k : ctx->kids) {
    (void)hipStreamSynchronize(k->stream);
    ms_ctx_destroy(k);
  }
  ctx->kids.clear();
  for (auto& v : ctx->prof)
    for (auto& r : v) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->sync_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->lu_ev) (void)hipEventDestroy(e);
  if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (!ctx->owns_status && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  for (void* p : ctx->ws)
    if (p) (void)hipFree(p);
  for (void* p : ctx->gws)
    if (p) (void)hipFree(p);
  if (ctx->owns_status && ctx->d_status) (void)hipFree(ctx->d_status);
  delete ctx;
  return MS_OK;
}

ms_status ms_ctx_sync(ms_ctx ctx) {
  if (!ctx) return MS_ERR_ARG;
  MS_HIP(ctx, hipSetDevice(ctx->device));
  MS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  int32_t st = 0;
  MS_HIP(ctx, hipMemcpy(&st, ctx->d_status, sizeof st, hipMemcpyDeviceToHost));
  MS_HIP(ctx, hipMemset(ctx->d_status, 0, sizeof(int32_t)));
  if (st != 0) return fail(ctx, (ms_status)st, "device reported %s", ms_status_str((ms_status)st));
  return MS_OK;
}

static const char* const kProfNames[PC_COUNT] = {"iface_gemm", "lu_panel", "lu_swap", "lu_update", "trsm",
                                                  "jacobi",     "prep_gemm", "elem", "other", "lu_inner"};

ms_status ms_debug_profile(ms_ctx ctx, uint32_t mask) {
  if (!ctx) return MS_ERR_ARG;
  std::vector<ms_ctx> all{ctx};
  for (size_t i = 0; i < all.size(); ++i) {
    all[i]->prof_mask = mask;
    for (ms_ctx k : all[i]->kids) all.push_back(k);
  }
  return MS_OK;
}

ms_status ms_debug_profile_read(ms_ctx ctx, const char* category, double* total_ms, int64_t* launches,
                                double* flops, double* bytes) {
  if (!ctx || !category || !total_ms || !launches || !flops || !bytes) return MS_ERR_ARG;
  int cat = -1;
  for (int i = 0; i < PC_COUNT; ++i)
    if (strcmp(category, kProfNames[i]) == 0) cat = i;
  if (cat < 0) return fail(ctx, MS_ERR_ARG, "unknown profiler category '%s'", category);
  MS_HIP(ctx, hipSetDevice(ctx->device));
  MS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  double tot = 0.0, fl = 0.0, by = 0.0;
  int64_t cnt = 0;
  std::vector<ms_ctx> all{ctx};   // the context and all its internal descendants
  for (size_t i = 0; i < all.size(); ++i)
    for (ms_ctx k : all[i]->kids) all.push_back(k);
  for (ms_ctx c : all) {
    MS_HIP(ctx, hipStreamSynchronize(c->stream));
    for (auto& r : c->prof[cat]) {
      float ms = 0.f;
      MS_HIP(ctx, hipEventElapsedTime(&ms, r.a, r.b));
      tot += ms;
      fl += r.flops;
      by += r.bytes;
      c->ev_pool.push_back(r.a);
      c->ev_pool.push_back(r.b);
    }
    cnt += (int64_t)c->prof[cat].size();
    c->prof[cat].clear();
  }
  *launches = cnt;
  *total_ms = tot;
  *flops = fl;
  *bytes = by;
  return MS_OK;
}

// ------------------------------------------------------------------------------------------
ms_status ms_slices_prepare(ms_ctx ctx, int64_t n_g, const int32_t* g_mn, const double* bvec, const double* kpar,
                            double vlead_left, double vlead_right, int64_t n_slices, int64_t n_q,
                            const int32_t* q_of_ij, const void* vq, ms_slices* inout) {
  if (!ctx) return MS_ERR_ARG;
  if (bad_ptr(g_mn) || bad_ptr(bvec) || bad_ptr(kpar) || bad_ptr(q_of_ij) || bad_ptr(vq))
    return fail(ctx, MS_ERR_ARG, "NULL input pointer");
  MS_TRY(check_slices(ctx, inout));
  if (inout->n_g != n_g || inout->n_slices != n_slices)
    return fail(ctx, MS_ERR_ARG, "inout sizes do not match n_g / n_slices");
  if (n_q <= 0) return fail(ctx, MS_ERR_ARG, "n_q must be positive");
  if (!std::isfinite(vlead_left) || !std::isfinite(vlead_right))
    return fail(ctx, MS_ERR_ARG, "lead potentials must be finite");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  const int n = (int)n_g;
  const int ns = (int)n_slices;
  const int64_t nn = (int64_t)n * n;
  double* eps = inout->eps;
  double2* ovl = c2(inout->ovl);

  void *kin, *shift, *W, *U;
  MS_TRY(workspace(ctx, WS_KIN, n * sizeof(double), &kin));
  MS_TRY(launch_kin_eps(ctx, n, g_mn, bvec, kpar, vlead_left, vlead_right, (double*)kin, eps,
                        eps + (int64_t)(ns + 1) * n));
  MS_TRY(launch_nonfinite_scan(ctx, (int64_t)ns * n_q, c2(vq), ctx->d_status));
  // every index of the difference map must address vq
  void* mm = nullptr;
  MS_TRY(workspace(ctx, WS_MISC, 4 * sizeof(int32_t), &mm));
  MS_TRY(launch_minmax(ctx, nn, q_of_ij, (int32_t*)mm));
  int32_t qr[3] = {0, 0, 0};
  MS_HIP(ctx, hipMemcpyAsync(qr, mm, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(qr + 2, q_of_ij, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  MS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (qr[0] < 0 || qr[1] >= n_q)
    return fail(ctx, MS_ERR_ARG, "q_of_ij values span [%d,%d], outside [0,%lld)", qr[0], qr[1], (long long)n_q);
  const int32_t q0 = qr[2];

  // Warm start: slices 0, S, 2S, ... are solved first from V = I; every slice is then
  // solved from V = the eigenvectors of its nearest such reference slice, which leaves
  // the one-sided Jacobi far fewer sweeps (adjacent slices differ by a thin layer).
  int S = WARM_STRIDE;
  if (const char* env = getenv("MS_EIG_WARM_STRIDE")) S = std::max(0, atoi(env));
  const bool warm = S > 1 && ns > S;
  const int nref = warm ? (ns + S - 1) / S : 0;
  const int nbuf = warm ? 4 : 3;
  int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(ns, (int64_t)(PREP_BUDGET / (nbuf * nn * sizeof(double2)))));
  chunk = std::min(chunk, 256);
  void *Z = nullptr, *V = nullptr, *Uref = nullptr;
  MS_TRY(workspace(ctx, WS_SHIFT, chunk * sizeof(double), &shift));
  MS_TRY(workspace(ctx, WS_W, (size_t)chunk * nn * sizeof(double2), &W));
  MS_TRY(workspace(ctx, WS_U, (size_t)(chunk + 1) * nn * sizeof(double2), &U));
  MS_TRY(workspace(ctx, WS_Z, (size_t)chunk * nn * sizeof(double2), &Z));
  if (warm) {
    MS_TRY(workspace(ctx, WS_PREP_V, (size_t)chunk * nn * sizeof(double2), &V));
    MS_TRY(workspace(ctx, WS_UREF, (size_t)nref * nn * sizeof(double2), &Uref));
  }
  double2* Ub = c2(U);
  // pass 1: the reference slices from V = I (their eps rows are rewritten by pass 2)
  for (int r0 = 0; r0 < nref; r0 += chunk) {
    const int bc = std::min(chunk, nref - r0);
    const double2* vq_r = c2(vq) + (int64_t)r0 * S * n_q;
    MS_TRY(launch_slice_shift(ctx, n, bc, (const double*)kin, n_q, (int64_t)S * n_q, vq_r, q0, (double*)shift));
    MS_TRY(launch_hgather(ctx, n, bc, (const double*)kin, (const double*)shift, (int64_t)S * n_q, vq_r, q_of_ij,
                          c2(W)));
    MS_TRY(launch_hgather(ctx, n, bc, (const double*)kin, nullptr, (int64_t)S * n_q, vq_r, q_of_ij, Ub + nn));
    MS_TRY(jacobi_eigh(ctx, n, bc, c2(W), Ub + nn, c2(Z), eps + (int64_t)(r0 * S + 1) * n, (int64_t)S * n,
                       c2(Uref) + (int64_t)r0 * nn, nn, ctx->d_status));
  }
  for (int s0 = 0; s0 < ns; s0 += chunk) {
    const int bc = std::min(chunk, ns - s0);
    const double2* vq_c = c2(vq) + (int64_t)s0 * n_q;
    MS_TRY(launch_slice_shift(ctx, n, bc, (const double*)kin, n_q, n_q, vq_c, q0, (double*)shift));
    MS_TRY(launch_hgather(ctx, n, bc, (const double*)kin, (const double*)shift, n_q, vq_c, q_of_ij, c2(W)));
    // H itself into U slots 1..bc (the eigenvectors overwrite it at the end)
    MS_TRY(launch_hgather(ctx, n, bc, (const double*)kin, nullptr, n_q, vq_c, q_of_ij, Ub + nn));
    double2* Wstart = c2(W);
    if (warm) {   // (H + cI) U_ref
      MS_TRY(launch_gather_ref(ctx, n, bc, s0, S, nref, c2(Uref), c2(Z)));
      GemmArgs g;
      g.M = n; g.N = n; g.K = n;
      g.A = W; g.lda = n; g.sA = nn;
      g.B = Z; g.ldb = n; g.sB = nn;
      g.C = c2(V); g.ldc = n; g.sC = nn;
      g.batch = bc;
      g.prof = PC_PREP_GEMM;
      MS_TRY(zgemm(ctx, g));
      Wstart = c2(V);
    }
    // slice s0+i (paper p = s0+i+1) -> eps row s0+i+1, U slot i+1
    MS_TRY(jacobi_eigh(ctx, n, bc, Wstart, Ub + nn, c2(Z), eps + (int64_t)(s0 + 1) * n, n, Ub + nn, nn,
                       ctx->d_status));
    // overlaps O^p = U^p^dagger U^{p+1}; slots: 0 = U^{s0} (previous chunk), i = U^{s0+i}
    const int P0 = s0 + 1, P1 = s0 + bc;
    if (P0 == 1) MS_TRY(launch_copy_boundary_overlaps(ctx, n, Ub + nn, ovl, 0));   // O^0 = U^1
    const int pstart = (P0 == 1) ? P0 : P0 - 1;
    if (P1 > pstart) {
      GemmArgs g;
      g.M = n; g.N = n; g.K = n;
      g.opA = OP_C; g.A = Ub + (int64_t)(pstart - P0 + 1) * nn; g.lda = n; g.sA = nn;
      g.opB = OP_N; g.B = Ub + (int64_t)(pstart - P0 + 2) * nn; g.ldb = n; g.sB = nn;
      g.C = ovl + (int64_t)pstart * nn; g.ldc = n; g.sC = nn;
      g.batch = P1 - pstart;
      g.prof = PC_PREP_GEMM;
      MS_TRY(zgemm(ctx, g));
    }
    if (inout->evec)
      MS_HIP(ctx, hipMemcpyAsync(c2(inout->evec) + (int64_t)s0 * nn, Ub + nn, (size_t)bc * nn * sizeof(double2),
                                 hipMemcpyDeviceToDevice, ctx->stream));
    MS_HIP(ctx, hipMemcpyAsync(Ub, Ub + (int64_t)bc * nn, nn * sizeof(double2), hipMemcpyDeviceToDevice,
                               ctx->stream));
  }
  // O^{n_slices} = U^{n_slices}^dagger
  MS_TRY(launch_copy_boundary_overlaps(ctx, n, Ub, ovl + (int64_t)ns * nn, 1));
  return MS_OK;
}

// ------------------------------------------------------------------------------------------
ms_status ms_slice_smatrix(ms_ctx ctx, const ms_slices* slices, double energy, int64_t p0, int64_t p1,
                           const ms_smat* out) {
  if (!ctx) return MS_ERR_ARG;
  MS_TRY(check_slices(ctx, slices));
  if (!std::isfinite(energy)) return fail(ctx, MS_ERR_ARG, "energy must be finite");
  if (p0 < 0 || p1 > slices->n_slices + 1 || p0 >= p1)
    return fail(ctx, MS_ERR_ARG, "interface range [%lld,%lld) outside [0,%lld]", (long long)p0, (long long)p1,
                (long long)slices->n_slices + 1);
  if (!out) return fail(ctx, MS_ERR_ARG, "out is NULL");
  for (int64_t i = 0; i < p1 - p0; ++i) MS_TRY(check_smat(ctx, out + i, slices->n_g, "out[i]"));
  MS_HIP(ctx, hipSetDevice(ctx->device));
  const int n = (int)slices->n_g, ns = (int)slices->n_slices, nrows = ns + 2;
  const int64_t nn = (int64_t)n * n;
  void *en, *kb, *pb, *aug, *xc, *yc, *z, *s4, *piv;
  MS_TRY(workspace(ctx, WS_EN, sizeof(double), &en));
  MS_TRY(upload(ctx, en, &energy, sizeof(double)));
  MS_TRY(workspace(ctx, WS_K, (size_t)nrows * n * sizeof(double2), &kb));
  MS_TRY(workspace(ctx, WS_P, (size_t)nrows * n * sizeof(double2), &pb));
  MS_TRY(launch_wavevectors(ctx, n, nrows, 1, slices->eps, (const double*)en, slices->dz, c2(kb), c2(pb)));
  const int64_t per = 10 * nn * (int64_t)sizeof(double2);
  int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(p1 - p0, (int64_t)(PREP_BUDGET / per)));
  chunk = std::min(chunk, 4096);
  MS_TRY(workspace(ctx, WS_AUG, (size_t)chunk * 3 * nn * sizeof(double2), &aug));
  MS_TRY(workspace(ctx, WS_XC, (size_t)chunk * nn * sizeof(double2), &xc));
  MS_TRY(workspace(ctx, WS_YC, (size_t)chunk * nn * sizeof(double2), &yc));
  MS_TRY(workspace(ctx, WS_Z, (size_t)chunk * 2 * nn * sizeof(double2), &z));
  MS_TRY(workspace(ctx, WS_S4, (size_t)chunk * 4 * nn * sizeof(double2), &s4));
  MS_TRY(workspace(ctx, WS_PIV, (size_t)chunk * n * sizeof(int32_t), &piv));
  for (int64_t q = p0; q < p1; q += chunk) {
    const int bc = (int)std::min<int64_t>(chunk, p1 - q);
    MS_TRY(launch_xy(ctx, n, bc, c2(slices->ovl), c2(kb), (int)q, c2(aug), c2(xc), c2(yc)));
    MS_TRY(getrf_aug(ctx, c2(aug), n, 3 * n, 3 * nn, bc, (int32_t*)piv, ctx->d_status, 0));
    MS_TRY(trsm_upper_aug(ctx, c2(aug), n, 3 * n, 3 * nn, bc, c2(z), 2 * n, 2 * nn, ctx->d_status, 0));
    double2* st = c2(s4);
    double2* srp = st + (int64_t)bc * nn;
    double2* sr = srp + (int64_t)bc * nn;
    double2* stp = sr + (int64_t)bc * nn;
    // S21 = Y X^-1
    GemmArgs g;
    g.M = n; g.N = n; g.K = n;
    g.A = yc; g.lda = n; g.sA = nn;
    g.B = z; g.ldb = 2 * n; g.sB = 2 * nn;
    g.C = sr; g.ldc = n; g.sC = nn;
    g.batch = bc;
    MS_TRY(zgemm(ctx, g));
    // Xc <- X - Y (X^-1 Y)
    g.B = c2(z) + n;
    g.C = c2(xc);
    g.alpha = MONE;
    g.beta = ONE;
    MS_TRY(zgemm(ctx, g));
    MS_TRY(launch_smat_finish(ctx, n, bc, c2(z), c2(xc), c2(pb), (int)q, st, srp, stp));
    for (int i = 0; i < bc; ++i) {
      const ms_smat& o = out[q - p0 + i];
      const size_t bytes = nn * sizeof(double2);
      MS_HIP(ctx, hipMemcpyAsync(o.t, st + i * nn, bytes, hipMemcpyDeviceToDevice, ctx->stream));
      MS_HIP(ctx, hipMemcpyAsync(o.rp, srp + i * nn, bytes, hipMemcpyDeviceToDevice, ctx->stream));
      MS_HIP(ctx, hipMemcpyAsync(o.r, sr + i * nn, bytes, hipMemcpyDeviceToDevice, ctx->stream));
      MS_HIP(ctx, hipMemcpyAsync(o.tp, stp + i * nn, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    }
  }
  return MS_OK;
}

// ------------------------------------------------------------------------------------------
namespace {

struct Blocks {
  double2 *t, *rp, *r, *tp;
};

// C = alpha A B + beta C for n x n operands A (lda), B (ldb), C (ldc); with fp32 the operands are
// rounded to complex64 and multiplied on FP32 MFMA with FP32 accumulation (alpha, beta and C
// stay FP64)
ms_status gemm_form(ms_ctx ctx, bool fp32, int n, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                    int64_t ldc, double2 alpha, double2 beta) {
  if (!fp32) return gemm(ctx, n, n, n, A, lda, OP_N, B, ldb, OP_N, C, ldc, alpha, beta);
  const int64_t ca = (int64_t)(n - 1) * lda + n, cb = (int64_t)(n - 1) * ldb + n;   // elements spanned
  void *a32, *b32;
  MS_TRY(workspace(ctx, WS_S32A, (size_t)ca * sizeof(float2), &a32));
  MS_TRY(workspace(ctx, WS_S32B, (size_t)cb * sizeof(float2), &b32));
  MS_TRY(launch_to_c64(ctx, ca, c2(A), static_cast<float2*>(a32)));
  MS_TRY(launch_to_c64(ctx, cb, c2(B), static_cast<float2*>(b32)));
  GemmArgs g;
  g.M = n; g.N = n; g.K = n;
  g.A = a32; g.lda = lda;
  g.B = b32; g.ldb = ldb;
  g.C = c2(C); g.ldc = ldc;
  g.alpha = alpha; g.beta = beta;
  return cgemm32(ctx, g);
}

// out = a * b (Redheffer star product); out must not alias a or b.  F = I - rp_a r_b, its LU
// and the solves with it are FP64 in both forms; with fp32 the six products that follow run on
// FP32 MFMA.
ms_status star(ms_ctx ctx, int n, Blocks a, Blocks b, Blocks out, bool fp32 = false) {
  const int64_t nn = (int64_t)n * n;
  void *aug, *z, *g, *h, *v, *piv;
  MS_TRY(workspace(ctx, WS_AUG, 3 * nn * sizeof(double2), &aug));
  MS_TRY(workspace(ctx, WS_Z, 2 * nn * sizeof(double2), &z));
  MS_TRY(workspace(ctx, WS_G, nn * sizeof(double2), &g));
  MS_TRY(workspace(ctx, WS_H, nn * sizeof(double2), &h));
  MS_TRY(workspace(ctx, WS_V, nn * sizeof(double2), &v));
  MS_TRY(workspace(ctx, WS_PIV, n * sizeof(int32_t), &piv));
  const size_t bytes = nn * sizeof(double2);
  // [F | t_a | rp_a] with F = I - rp_a r_b
  MS_TRY(launch_star_aug(ctx, n, a.t, a.rp, c2(aug)));
  MS_TRY(gemm(ctx, n, n, n, a.rp, n, OP_N, b.r, n, OP_N, aug, 3 * n, MONE, ONE));
  MS_TRY(getrf_aug(ctx, c2(aug), n, 3 * n, 3 * nn, 1, (int32_t*)piv, ctx->d_status, 0));
  // Z = [F^-1 t_a | F^-1 rp_a]
  MS_TRY(trsm_upper_aug(ctx, c2(aug), n, 3 * n, 3 * nn, 1, c2(z), 2 * n, 2 * nn, ctx->d_status, 0));
  const double2* w1 = c2(z);
  const double2* w2 = c2(z) + n;
  // G = tp_a r_b
  MS_TRY(gemm_form(ctx, fp32, n, a.tp, n, b.r, n, g, n, ONE, ZERO));
  // t = t_b W1
  MS_TRY(gemm_form(ctx, fp32, n, b.t, n, w1, 2 * n, out.t, n, ONE, ZERO));
  // r = r_a + G W1
  MS_HIP(ctx, hipMemcpyAsync(out.r, a.r, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  MS_TRY(gemm_form(ctx, fp32, n, g, n, w1, 2 * n, out.r, n, ONE, ONE));
  // rp = rp_b + (t_b W2) tp_b
  MS_TRY(gemm_form(ctx, fp32, n, b.t, n, w2, 2 * n, h, n, ONE, ZERO));
  MS_HIP(ctx, hipMemcpyAsync(out.rp, b.rp, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  MS_TRY(gemm_form(ctx, fp32, n, h, n, b.tp, n, out.rp, n, ONE, ONE));
  // tp = (tp_a + G W2) tp_b
  MS_HIP(ctx, hipMemcpyAsync(v, a.tp, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  MS_TRY(gemm_form(ctx, fp32, n, g, n, w2, 2 * n, v, n, ONE, ONE));
  MS_TRY(gemm_form(ctx, fp32, n, v, n, b.tp, n, out.tp, n, ONE, ZERO));
  return MS_OK;
}

Blocks blocks_of(const ms_smat& s) { return Blocks{c2(s.t), c2(s.rp), c2(s.r), c2(s.tp)}; }

}  // namespace

// ------------------------------------------------------------------------------------------
// First variation of T with respect to the slice potentials.
//
// dt_ij = (1/(2 i k_i)) int phi_i^dagger dH psi_j dz (psi_j: incident from the left in open
// channel j; phi_i: outgoing only into the right lead's open channel i), dT = sum_ij (k_i/k_j)
// 2 Re(conj(t_ij) dt_ij).  Both states' amplitudes (A^p, B^p) at the reference plane of slice p
// come from the left cascade L = S(0,p) and the right cascade R = S(p,N+1):
// (I - L12 R21) A^p = L11 A^0 + L12 R22 B^{N+1}, B^p = R21 A^p + R22 B^{N+1}.  The right
// cascades are swept once from the right lead, kept at every `ck`-th plane and recomputed
// segment by segment while the left cascade is swept from the left lead.
namespace {

ms_status check_energies(ms_ctx ctx, int64_t count, const double* energies);
ms_status sync_events(ms_ctx ctx, size_t count);

struct GradHost {   // the slices' thicknesses and the two leads' channel energies, on the host
  std::vector<double> dz, el, er;
};

ms_status grad_host(ms_ctx ctx, const ms_slices* sl, GradHost* h) {
  const int n = (int)sl->n_g, ns = (int)sl->n_slices;
  h->dz.resize(ns);
  h->el.resize(n);
  h->er.resize(n);
  MS_HIP(ctx, hipMemcpyAsync(h->dz.data(), sl->dz, ns * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(h->el.data(), sl->eps, n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(h->er.data(), sl->eps + (int64_t)(ns + 1) * n, n * sizeof(double),
                             hipMemcpyDeviceToHost, ctx->stream));
  MS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return MS_OK;
}

int open_count(const std::vector<double>& eps, double energy) {
  int c = 0;
  for (double x : eps) c += x < energy;
  return c;
}

Blocks blk(double2* base, int64_t nn) { return Blocks{base, base + nn, base + 2 * nn, base + 3 * nn}; }

// The energies of one batch go through every launch together: matrix b of a batched operand
// sits b * stride elements after matrix 0.  Channel tables are padded with -1 to the batch's
// largest open counts NL, NR; padded columns of the reduced states stay zero throughout.
struct Batch {
  ms_ctx ctx;
  int nb;
};

ms_status gemmb(const Batch& B, int M, int N, int K, const double2* A, int64_t lda, int64_t sA, const double2* X,
                int64_t ldx, int64_t sX, int opX, double2* C, int64_t ldc, int64_t sC, double2 alpha, double2 beta) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.sA = sA;
  g.B = X; g.ldb = ldx; g.sB = sX; g.opB = opX;
  g.C = C; g.ldc = ldc; g.sC = sC;
  g.alpha = alpha; g.beta = beta;
  g.batch = B.nb;
  return zgemm(B.ctx, g);
}

ms_status copyb(const Batch& B, int nrow, int ncol, const double2* src, int64_t lds, int64_t ss, double2* dst,
                int64_t ldd, int64_t sd) {
  return launch_gather2(B.ctx, nrow, ncol, nullptr, nullptr, src, lds, dst, ldd, B.nb, 0, 0, ss, sd);
}

// Reduced cascade states (row-major, c128), one per energy, `s` elements apart:
//   right, R = S(p, N+1): r (n x n), tpc = t'[:, orr] (n x NR), trow = t[orr, :] (NR x n),
//                         rpo = r'[orr, orr] (NR x NR)
//   left,  L = S(0, p):   rp = r' (n x n), ltc = t[:, ol] (n x NL)
// which is all the amplitudes and the whole S's open blocks need.  Their star products with
// a slice S cost 4 1/3 n^3 complex MACs instead of 10 1/3 for all four blocks.
struct RState {
  double2 *r, *tpc, *trow, *rpo;
  int64_t s;
};
struct LState {
  double2 *rp, *ltc;
  int64_t s;
};

int64_t rstate_size(int n, int nr) { return (int64_t)n * n + 2 * (int64_t)n * nr + (int64_t)nr * nr; }
RState rstate(double2* base, int n, int nr) {
  const int64_t nn = (int64_t)n * n;
  return RState{base, base + nn, base + nn + (int64_t)n * nr, base + nn + 2 * (int64_t)n * nr, rstate_size(n, nr)};
}
int64_t lstate_size(int n, int nl) { return (int64_t)n * n + (int64_t)n * nl; }
LState lstate(double2* base, int n, int nl) { return LState{base, base + (int64_t)n * n, lstate_size(n, nl)}; }

struct GradWork {   // scratch of the reduced star products, per energy: aug, w, tmp, thin, piv
  double2 *aug, *w, *tmp, *thin;
  int64_t sg, sw, st;   // strides of aug, w and thin (tmp: n * n)
  int32_t* piv;
};

// out = a * b with a = S(p,p+1) (full blocks, energies sa apart), b = S(p+1,N+1) (reduced);
// F = I - rp_a r_b, W = F^-1 [t_a | rp_a tpc_b]:  r = r_a + tp_a r_b W_t,
// tpc = tp_a (tpc_b + r_b W_x), trow = trow_b W_t,  rpo = rpo_b + trow_b W_x.
ms_status rstar(const Batch& B, int n, int nr, Blocks a, int64_t sa, RState b, RState out, const GradWork& g) {
  ms_ctx ctx = B.ctx;
  const int64_t nn = (int64_t)n * n;
  const int ld = 2 * n + nr, wl = n + nr;
  MS_TRY(launch_eye(ctx, n, ld, g.aug, B.nb, g.sg));
  MS_TRY(gemmb(B, n, n, n, a.rp, n, sa, b.r, n, b.s, OP_N, g.aug, ld, g.sg, MONE, ONE));
  MS_TRY(copyb(B, n, n, a.t, n, sa, g.aug + n, ld, g.sg));
  if (nr > 0) MS_TRY(gemmb(B, n, nr, n, a.rp, n, sa, b.tpc, nr, b.s, OP_N, g.aug + 2 * n, ld, g.sg, ONE, ZERO));
  MS_TRY(getrf_aug(ctx, g.aug, n, ld, g.sg, B.nb, g.piv, ctx->d_status, 0));
  MS_TRY(trsm_upper_aug(ctx, g.aug, n, ld, g.sg, B.nb, g.w, wl, g.sw, ctx->d_status, 0));
  const double2* wt = g.w;
  const double2* wx = g.w + n;
  MS_TRY(gemmb(B, n, n, n, b.r, n, b.s, wt, wl, g.sw, OP_N, g.tmp, n, nn, ONE, ZERO));
  MS_TRY(copyb(B, n, n, a.r, n, sa, out.r, n, out.s));
  MS_TRY(gemmb(B, n, n, n, a.tp, n, sa, g.tmp, n, nn, OP_N, out.r, n, out.s, ONE, ONE));
  if (nr > 0) {
    MS_TRY(copyb(B, n, nr, b.tpc, nr, b.s, g.thin, nr, g.st));
    MS_TRY(gemmb(B, n, nr, n, b.r, n, b.s, wx, wl, g.sw, OP_N, g.thin, nr, g.st, ONE, ONE));
    MS_TRY(gemmb(B, n, nr, n, a.tp, n, sa, g.thin, nr, g.st, OP_N, out.tpc, nr, out.s, ONE, ZERO));
    MS_TRY(gemmb(B, nr, n, n, b.trow, n, b.s, wt, wl, g.sw, OP_N, out.trow, n, out.s, ONE, ZERO));
    MS_TRY(copyb(B, nr, nr, b.rpo, nr, b.s, out.rpo, nr, out.s));
    MS_TRY(gemmb(B, nr, nr, n, b.trow, n, b.s, wx, wl, g.sw, OP_N, out.rpo, nr, out.s, ONE, ONE));
  }
  return MS_OK;
}

// out = a * b with a = S(0,p) (reduced), b = S(p,p+1) (full blocks, energies sb apart);
// F = I - rp_a r_b, W = F^-1 [rp_a | ltc_a]:  rp = rp_b + (t_b W_rp) tp_b,  ltc = t_b W_l.
ms_status lstar(const Batch& B, int n, int nl, LState a, Blocks b, int64_t sb, LState out, const GradWork& g) {
  ms_ctx ctx = B.ctx;
  const int64_t nn = (int64_t)n * n;
  const int ld = 2 * n + nl, wl = n + nl;
  MS_TRY(launch_eye(ctx, n, ld, g.aug, B.nb, g.sg));
  MS_TRY(gemmb(B, n, n, n, a.rp, n, a.s, b.r, n, sb, OP_N, g.aug, ld, g.sg, MONE, ONE));
  MS_TRY(copyb(B, n, n, a.rp, n, a.s, g.aug + n, ld, g.sg));
  if (nl > 0) MS_TRY(copyb(B, n, nl, a.ltc, nl, a.s, g.aug + 2 * n, ld, g.sg));
  MS_TRY(getrf_aug(ctx, g.aug, n, ld, g.sg, B.nb, g.piv, ctx->d_status, 0));
  MS_TRY(trsm_upper_aug(ctx, g.aug, n, ld, g.sg, B.nb, g.w, wl, g.sw, ctx->d_status, 0));
  MS_TRY(gemmb(B, n, n, n, b.t, n, sb, g.w, wl, g.sw, OP_N, g.tmp, n, nn, ONE, ZERO));
  MS_TRY(copyb(B, n, n, b.rp, n, sb, out.rp, n, out.s));
  MS_TRY(gemmb(B, n, n, n, g.tmp, n, nn, b.tp, n, sb, OP_N, out.rp, n, out.s, ONE, ONE));
  if (nl > 0) MS_TRY(gemmb(B, n, nl, n, b.t, n, sb, g.w + n, wl, g.sw, OP_N, out.ltc, nl, out.s, ONE, ZERO));
  return MS_OK;
}

// the reduced right state of one slice S(p,p+1) (the cascade's first factor, p = N);
// ort: [nb][nr] right-lead channel table
ms_status rstate_of(const Batch& B, int n, int nr, const int32_t* ort, Blocks s, int64_t ss, RState out) {
  MS_TRY(copyb(B, n, n, s.r, n, ss, out.r, n, out.s));
  MS_TRY(launch_gather2(B.ctx, n, nr, nullptr, ort, s.tp, n, out.tpc, nr, B.nb, 0, nr, ss, out.s));
  MS_TRY(launch_gather2(B.ctx, nr, n, ort, nullptr, s.t, n, out.trow, n, B.nb, nr, 0, ss, out.s));
  return launch_gather2(B.ctx, nr, nr, ort, ort, s.rp, n, out.rpo, nr, B.nb, nr, nr, ss, out.s);
}

// channel counts of an energy batch and the bytes of device memory it needs
struct GradDims {
  int NL, NR;
};
GradDims grad_dims(const GradHost& h, int nb, const double* energy) {
  GradDims d{0, 0};
  for (int e = 0; e < nb; ++e) {
    d.NL = std::max(d.NL, open_count(h.el, energy[e]));
    d.NR = std::max(d.NR, open_count(h.er, energy[e]));
  }
  return d;
}
// planes per segment of slice S-matrices: the checkpoint spacing (the right cascades of a
// segment are recomputed from the checkpoint above it), or 16 when every plane is kept
int seg_planes(int ck) { return ck == 1 ? 16 : ck; }
int64_t grad_elems_per_energy(int n, int ns, int ck, GradDims d) {   // c128 elements
  const int64_t nn = (int64_t)n * n, rsz = rstate_size(n, d.NR), lsz = lstate_size(n, d.NL);
  const int64_t wmax = std::max(1, std::max(d.NL, d.NR)), m = d.NL + d.NR, wa = m;
  const int64_t nck = (ns + 1) / ck + 1;
  return (seg_planes(ck) + 1) * 4 * nn + nck * rsz + (ck + 2) * rsz + 2 * lsz + 2 * (int64_t)(ns + 2) * n +
         n * (2 * n + wmax) + n * (n + wmax) + nn + n * wmax + nn + m * (m + d.NR) + m * d.NR + n * (n + wa) +
         n * wa + 2 * n * (int64_t)d.NR + 3 * n * (int64_t)d.NL + 2 * nn;
}

// the gradient at nb energies, all on ctx's stream; grad: [nb][ns][n_q] c128
ms_status dT_dV_batch(ms_ctx ctx, const ms_slices* slices, const GradHost& h, int nb, const double* energy,
                      const int32_t* q_of_ij, int64_t n_q, int ck, double2* grad, double* t_r, int64_t* n_open) {
  const int n = (int)slices->n_g, ns = (int)slices->n_slices, nrows = ns + 2;
  const int64_t nn = (int64_t)n * n, s4 = 4 * nn;
  const Batch B{ctx, nb};
  const GradDims dims = grad_dims(h, nb, energy);
  const int NL = dims.NL, NR = dims.NR;
  // channel tables: ol [nb][NL] then orr [nb][NR], padded with -1
  std::vector<int32_t> tab((size_t)nb * (NL + NR), -1);
  for (int e = 0; e < nb; ++e) {
    int c = 0;
    for (int i = 0; i < n; ++i)
      if (h.el[i] < energy[e]) tab[(size_t)e * NL + c++] = i;
    c = 0;
    for (int i = 0; i < n; ++i)
      if (h.er[i] < energy[e]) tab[(size_t)nb * NL + (size_t)e * NR + c++] = i;
  }
  MS_HIP(ctx, hipMemsetAsync(grad, 0, (size_t)nb * ns * n_q * sizeof(double2), ctx->stream));
  const int64_t rsz = rstate_size(n, NR), lsz = lstate_size(n, NL);
  const int nck = (ns + 1) / ck + 1;            // planes 0, ck, 2 ck, ... <= ns
  const int wmax = std::max(1, std::max(NL, NR));
  const size_t E = sizeof(double2);
  void *seg, *cks, *rseg, *lb, *kb, *pb, *chd, *en, *aug, *w, *tmp, *thin, *tf, *pv;
  const int L = seg_planes(ck);
  MS_TRY(workspace(ctx, WS_GSEG, (size_t)(L + 1) * nb * s4 * E, &seg));
  MS_TRY(workspace(ctx, WS_GCK, (size_t)nck * nb * rsz * E, &cks));
  MS_TRY(workspace(ctx, WS_GRS, (size_t)(ck + 2) * nb * rsz * E, &rseg));
  MS_TRY(workspace(ctx, WS_GL, 2 * (size_t)nb * lsz * E, &lb));
  MS_TRY(workspace(ctx, WS_GK, (size_t)nb * nrows * n * E, &kb));
  MS_TRY(workspace(ctx, WS_GP, (size_t)nb * nrows * n * E, &pb));
  MS_TRY(workspace(ctx, WS_GCH, std::max<size_t>(1, tab.size()) * sizeof(int32_t), &chd));
  MS_TRY(workspace(ctx, WS_GEN, (size_t)nb * sizeof(double), &en));
  MS_TRY(workspace(ctx, WS_GAUG, (size_t)nb * n * (2 * n + wmax) * E, &aug));
  MS_TRY(workspace(ctx, WS_GY, (size_t)nb * n * (n + wmax) * E, &w));
  MS_TRY(workspace(ctx, WS_GT1, (size_t)nb * nn * E, &tmp));
  MS_TRY(workspace(ctx, WS_GBF, (size_t)nb * n * wmax * E, &thin));
  MS_TRY(workspace(ctx, WS_GMC, (size_t)nb * nn * E, &tf));
  MS_TRY(workspace(ctx, WS_GPIV, (size_t)nb * std::max(n, NL + NR) * sizeof(int32_t), &pv));
  if (!tab.empty()) MS_TRY(upload(ctx, chd, tab.data(), tab.size() * sizeof(int32_t)));
  MS_TRY(upload(ctx, en, energy, nb * sizeof(double)));
  const int64_t sk = (int64_t)nrows * n;
  MS_TRY(launch_wavevectors(ctx, n, nrows, nb, slices->eps, (const double*)en, slices->dz, c2(kb), c2(pb), sk));
  const int32_t* olt = (const int32_t*)chd;
  const int32_t* ort = olt + (int64_t)nb * NL;
  const GradWork gw{c2(aug), c2(w), c2(tmp), c2(thin), (int64_t)n * (2 * n + wmax), (int64_t)n * (n + wmax),
                    (int64_t)n * wmax, (int32_t*)pv};
  double2* segp = c2(seg);
  // S(p,p+1) for p in [p0,p1) and every energy: slot i = p - p0 holds energy e at (i nb + e) 4 n^2
  auto smats = [&](int p0, int p1) -> ms_status {
    std::vector<ms_smat> out(p1 - p0);
    for (int e = 0; e < nb; ++e) {
      for (int i = 0; i < p1 - p0; ++i) {
        double2* b = segp + ((int64_t)i * nb + e) * s4;
        out[i] = ms_smat{n, b, b + nn, b + 2 * nn, b + 3 * nn};
      }
      MS_TRY(ms_slice_smatrix(ctx, slices, energy[e], p0, p1, out.data()));
    }
    return MS_OK;
  };
  auto slot = [&](int i) { return blk(segp + (int64_t)i * nb * s4, nn); };

  // 1. right sweep R_p = S(p,p+1) * R_{p+1} from R_ns = S(ns,ns+1) (reduced); R_p kept when p % ck == 0
  double2* ckp = c2(cks);
  double2* racc[2] = {c2(rseg), c2(rseg) + (int64_t)nb * rsz};
  int cur = 0;
  for (int hi = ns; hi >= 0; hi -= (L + 1)) {   // chunks of up to L + 1 slice S-matrices
    const int lo = std::max(0, hi - L);
    MS_TRY(smats(lo, hi + 1));
    for (int p = hi; p >= lo; --p) {
      const Blocks sp = slot(p - lo);
      if (p == ns) {
        MS_TRY(rstate_of(B, n, NR, ort, sp, s4, rstate(racc[cur], n, NR)));
      } else {
        MS_TRY(rstar(B, n, NR, sp, s4, rstate(racc[cur], n, NR), rstate(racc[cur ^ 1], n, NR), gw));
        cur ^= 1;
      }
      if (p % ck == 0)
        MS_HIP(ctx, hipMemcpyAsync(ckp + (int64_t)(p / ck) * nb * rsz, racc[cur], (size_t)nb * rsz * E,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    }
  }
  // 2. the whole S = R_0 (its open blocks): T, R, N_open of each energy
  const RState whole = rstate(ckp, n, NR);
  MS_HIP(ctx, hipMemsetAsync(tf, 0, (size_t)nb * nn * E, ctx->stream));
  for (int e = 0; e < nb; ++e) {
    double2* te = c2(tf) + e * nn;
    MS_TRY(launch_scatter_rows(ctx, NR, n, ort + (int64_t)e * NR, whole.trow + e * rsz, te));   // t, open rows
    MS_TRY(launch_whole_T(ctx, n, energy[e], te, whole.r + e * rsz, slices->eps,
                          slices->eps + (int64_t)(ns + 1) * n, t_r + 2 * e, t_r + 2 * e + 1, n_open + e,
                          ctx->d_status));
  }
  if (NL == 0 || NR == 0) return MS_OK;       // no open channel at any energy: dT = 0
  // 3. incoming amplitudes of the out-states: [r_OO t'_OR; t_RO r'_RR] [x; y] = [0; e_i]
  //    (padded channels: identity rows and zero right-hand sides)
  const int m = NL + NR, mw = m + NR;
  void *os, *xs;
  MS_TRY(workspace(ctx, WS_GOS, (size_t)nb * m * mw * E, &os));
  MS_TRY(workspace(ctx, WS_GX, (size_t)nb * m * NR * E, &xs));
  MS_TRY(launch_grad_open_system(ctx, n, NL, NR, olt, ort, whole.r, whole.tpc, whole.trow, whole.rpo, rsz, c2(os),
                                 nb));
  MS_TRY(getrf_aug(ctx, c2(os), m, mw, (int64_t)m * mw, nb, (int32_t*)pv, ctx->d_status, 0));
  MS_TRY(trsm_upper_aug(ctx, c2(os), m, mw, (int64_t)m * mw, nb, c2(xs), NR, (int64_t)m * NR, ctx->d_status, 0));
  const int64_t sx = (int64_t)m * NR;
  const double2* xtop = c2(xs);                       // incoming from the left on ol (NL x NR)
  const double2* xbot = c2(xs) + (int64_t)NL * NR;    // incoming from the right on orr (NR x NR)
  // 4. segments of planes [lo, hi], lo >= 1: recompute R_p there, sweep L_p, add each slice
  const int wa = NL + NR, ldaug = n + wa;
  const int64_t sa2 = (int64_t)n * ldaug, sy = (int64_t)n * wa, snr = (int64_t)n * NR, snl = (int64_t)n * NL;
  void *aug2, *ys, *t1, *bps, *bph, *p1, *p2, *yg, *kc;
  MS_TRY(workspace(ctx, WS_GA2, (size_t)nb * sa2 * E, &aug2));
  MS_TRY(workspace(ctx, WS_GB2, (size_t)nb * sy * E, &ys));
  MS_TRY(workspace(ctx, WS_GFA, (size_t)nb * snr * E, &t1));
  MS_TRY(workspace(ctx, WS_GBP, (size_t)nb * snl * E, &bps));
  MS_TRY(workspace(ctx, WS_GFB, (size_t)nb * snr * E, &bph));
  MS_TRY(workspace(ctx, WS_GP1, (size_t)nb * snl * E, &p1));
  MS_TRY(workspace(ctx, WS_GP2, (size_t)nb * snl * E, &p2));
  MS_TRY(workspace(ctx, WS_GYG, (size_t)nb * nn * E, &yg));
  MS_TRY(workspace(ctx, WS_GKC, (size_t)nb * nn * E, &kc));
  double2* mc = c2(tf);   // t with its open rows is no longer needed
  double2* lbuf[2] = {c2(lb), c2(lb) + (int64_t)nb * lsz};
  int lc = 0;
  // segments [lo, hi]: with checkpoints every ck > 1 planes, hi + 1 is a checkpoint (or hi = ns);
  // with every plane kept (ck = 1), L planes each
  std::vector<double2*> rptr(L);
  for (int lo = 1; lo <= ns;) {
    const int hi = ck == 1 ? std::min(ns, lo + L - 1) : std::min(ns, (lo / ck + 1) * ck - 1);
    bool recompute = false;   // a plane of the segment without a stored right cascade
    for (int p = lo; p <= hi; ++p) recompute = recompute || p % ck != 0;
    // interfaces S(p,p+1), p in [lo-1, hi] (p < hi without a recompute): slot i = S(lo-1+i, lo+i)
    MS_TRY(smats(lo - 1, recompute ? hi + 1 : hi));
    // R_p for p = hi..lo: stored ones from their checkpoint, the others recomputed into rseg
    // slot p - lo from the one above (R_hi from the checkpoint at hi + 1, or S(ns,ns+1))
    double2* rs = c2(rseg);
    for (int p = hi; p >= lo; --p) {
      if (p % ck == 0) {
        rptr[p - lo] = ckp + (int64_t)(p / ck) * nb * rsz;
        continue;
      }
      const Blocks sp = slot(p - lo + 1);
      double2* dst = rs + (int64_t)(p - lo) * nb * rsz;
      if (p == ns) {
        MS_TRY(rstate_of(B, n, NR, ort, sp, s4, rstate(dst, n, NR)));
      } else {
        double2* right = (p == hi) ? ckp + (int64_t)((hi + 1) / ck) * nb * rsz : rptr[p + 1 - lo];
        MS_TRY(rstar(B, n, NR, sp, s4, rstate(right, n, NR), rstate(dst, n, NR), gw));
      }
      rptr[p - lo] = dst;
    }
    for (int p = lo; p <= hi; ++p) {
      // L_p = L_{p-1} * S(p-1,p)  (L_1 = S(0,1))
      const Blocks sprev = slot(p - lo);
      if (p == 1) {
        const LState l1 = lstate(lbuf[lc], n, NL);
        MS_TRY(copyb(B, n, n, sprev.rp, n, s4, l1.rp, n, l1.s));
        MS_TRY(launch_gather2(ctx, n, NL, nullptr, olt, sprev.t, n, l1.ltc, NL, nb, 0, NL, s4, l1.s));
      } else {
        MS_TRY(lstar(B, n, NL, lstate(lbuf[lc], n, NL), sprev, s4, lstate(lbuf[lc ^ 1], n, NL), gw));
        lc ^= 1;
      }
      const LState L = lstate(lbuf[lc], n, NL);
      const RState R = rstate(rptr[p - lo], n, NR);
      // [I - L12 R21 | L11[:, ol] | L11[:, ol] x_top + L12 (R22[:, orr] x_bot)]
      MS_TRY(launch_eye(ctx, n, ldaug, c2(aug2), nb, sa2));
      MS_TRY(gemmb(B, n, n, n, L.rp, n, L.s, R.r, n, R.s, OP_N, c2(aug2), ldaug, sa2, MONE, ONE));
      MS_TRY(copyb(B, n, NL, L.ltc, NL, L.s, c2(aug2) + n, ldaug, sa2));
      MS_TRY(gemmb(B, n, NR, NR, R.tpc, NR, R.s, xbot, NR, sx, OP_N, c2(t1), NR, snr, ONE, ZERO));
      MS_TRY(gemmb(B, n, NR, NL, L.ltc, NL, L.s, xtop, NR, sx, OP_N, c2(aug2) + n + NL, ldaug, sa2, ONE, ZERO));
      MS_TRY(gemmb(B, n, NR, n, L.rp, n, L.s, c2(t1), NR, snr, OP_N, c2(aug2) + n + NL, ldaug, sa2, ONE, ONE));
      MS_TRY(getrf_aug(ctx, c2(aug2), n, ldaug, sa2, nb, (int32_t*)pv, ctx->d_status, 0));
      MS_TRY(trsm_upper_aug(ctx, c2(aug2), n, ldaug, sa2, nb, c2(ys), wa, sy, ctx->d_status, 0));
      const double2* apsi = c2(ys);          // n x NL, ld wa
      const double2* aphi = c2(ys) + NL;     // n x NR, ld wa
      // B^p: psi: R21 a; phi: R21 a + R22 fb
      MS_TRY(gemmb(B, n, NL, n, R.r, n, R.s, apsi, wa, sy, OP_N, c2(bps), NL, snl, ONE, ZERO));
      MS_TRY(copyb(B, n, NR, c2(t1), NR, snr, c2(bph), NR, snr));
      MS_TRY(gemmb(B, n, NR, n, R.r, n, R.s, aphi, wa, sy, OP_N, c2(bph), NR, snr, ONE, ONE));
      // slice p: conj(M), then conj(K) = U conj(M) U^dagger, then g[q(a,b)] += K_ab
      MS_TRY(launch_grad_p(ctx, n, NL, NR, aphi, wa, sy, c2(bph), NR, snr, whole.trow, rsz, olt, NL, c2(kb), sk,
                           c2(p1), c2(p2), snl, nb));
      MS_TRY(launch_grad_m(ctx, n, NL, c2(kb) + (int64_t)p * n, sk, h.dz[p - 1], c2(p1), c2(p2), snl, apsi, wa, sy,
                           c2(bps), NL, snl, mc, nn, nb));
      const double2* U = c2(slices->evec) + (int64_t)(p - 1) * nn;
      MS_TRY(gemmb(B, n, n, n, mc, n, nn, U, n, 0, OP_C, c2(yg), n, nn, ONE, ZERO));
      MS_TRY(gemmb(B, n, n, n, U, n, 0, c2(yg), n, nn, OP_N, c2(kc), n, nn, ONE, ZERO));
      MS_TRY(launch_grad_scatter(ctx, nn, q_of_ij, c2(kc), nn, reinterpret_cast<double*>(grad) + 2 * (int64_t)(p - 1) * n_q,
                                 2 * (int64_t)ns * n_q, nb));
    }
    lo = hi + 1;
  }
  return MS_OK;
}

}  // namespace

ms_status ms_dT_dV(ms_ctx ctx, const ms_slices* slices, int64_t n_e, const double* energies, const int32_t* q_of_ij,
                   int64_t n_q, int64_t checkpoint, void* grad, double* t_r, int64_t* n_open) {
  if (!ctx) return MS_ERR_ARG;
  MS_TRY(check_slices(ctx, slices));
  if (bad_ptr(slices->evec)) return fail(ctx, MS_ERR_ARG, "slices->evec (the eigenvectors) is required");
  if (n_e < 0) return fail(ctx, MS_ERR_ARG, "n_e must be >= 0");
  if (n_e == 0) return MS_OK;
  if (bad_ptr(energies) || bad_ptr(q_of_ij) || bad_ptr(grad) || bad_ptr(t_r) || bad_ptr(n_open))
    return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  MS_TRY(check_energies(ctx, n_e, energies));
  if (n_q < 1) return fail(ctx, MS_ERR_ARG, "n_q must be >= 1");
  if (checkpoint < 0) return fail(ctx, MS_ERR_ARG, "checkpoint must be >= 0");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  const int n = (int)slices->n_g, ns = (int)slices->n_slices;
  const int64_t nn = (int64_t)n * n;
  {   // every q_of_ij value must index the gradient's n_q columns (they are scatter targets)
    void* mm;
    MS_TRY(workspace(ctx, WS_MISC, 4 * sizeof(int32_t), &mm));
    MS_TRY(launch_minmax(ctx, nn, q_of_ij, (int32_t*)mm));
    int32_t qr[2] = {0, 0};
    MS_HIP(ctx, hipMemcpyAsync(qr, mm, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    MS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (qr[0] < 0 || qr[1] >= n_q)
      return fail(ctx, MS_ERR_ARG, "q_of_ij values span [%d,%d], outside [0,%lld)", qr[0], qr[1], (long long)n_q);
  }
  GradHost h;
  MS_TRY(grad_host(ctx, slices, &h));
  // Energies are split over up to three internal contexts (own stream and workspace, forked
  // from and joined to the caller's stream, each driven by a host thread of its own, since the
  // segments' host steps wait for their stream); each context's energies go through every
  // launch together, as many per batch as its share of 3/4 of the free device memory holds
  // (at most 16).  One energy alone leaves most of the chip idle in its single-matrix LU and
  // GEMM steps: the streams overlap one energy's LU with another's GEMMs, the batches fill both.
  const int nrun = n_e > 1 ? (int)std::min<int64_t>(3, n_e) : 0;
  const int64_t R = std::max(1, nrun);
  size_t free_b = 0, total_b = 0;
  MS_HIP(ctx, hipMemGetInfo(&free_b, &total_b));
  const GradDims all = grad_dims(h, (int)n_e, energies);
  // checkpoint 0: every plane's right cascade kept (none recomputed) when that fits the energies
  // in flight into 3/4 of the free device memory, else about sqrt(N_s + 1) planes apart
  const int64_t budget = (int64_t)(free_b / 4) * 3;
  int ck = (int)std::min<int64_t>(checkpoint, ns + 1);
  if (checkpoint == 0) {
    const int64_t inflight = std::min<int64_t>(n_e, 16 * R);
    const int64_t all_planes = grad_elems_per_energy(n, ns, 1, all) * (int64_t)sizeof(double2) * inflight;
    ck = all_planes <= budget ? 1 : std::max(1, (int)std::lround(std::sqrt((double)(ns + 1))));
  }
  const int64_t per_e = grad_elems_per_energy(n, ns, ck, all) * (int64_t)sizeof(double2);
  const int64_t fit = std::max<int64_t>(1, budget / R / std::max<int64_t>(1, per_e));
  std::vector<ms_ctx> run(R, ctx);
  for (int r = 0; r < nrun; ++r) MS_TRY(child(ctx, r, &run[r]));
  if (nrun > 0) {
    MS_TRY(sync_events(ctx, 1 + nrun));
    MS_HIP(ctx, hipEventRecord(ctx->sync_ev[0], ctx->stream));
    for (int r = 0; r < nrun; ++r) MS_HIP(ctx, hipStreamWaitEvent(run[r]->stream, ctx->sync_ev[0], 0));
  }
  auto energies_of = [&](int r) -> ms_status {   // context r: energies [r n_e / R, (r+1) n_e / R)
    const int64_t eb = r * n_e / R, cnt = (r + 1) * n_e / R - eb;
    const int64_t cap = std::min<int64_t>({cnt, 16, fit});
    const int64_t nbat = (cnt + cap - 1) / cap;
    for (int64_t b = 0; b < nbat; ++b) {   // batches of near-equal size
      const int64_t e0 = eb + b * cnt / nbat, e1 = eb + (b + 1) * cnt / nbat;
      MS_TRY(dT_dV_batch(run[r], slices, h, (int)(e1 - e0), energies + e0, q_of_ij, n_q, ck,
                         static_cast<double2*>(grad) + e0 * (int64_t)ns * n_q, t_r + 2 * e0, n_open + e0));
    }
    return MS_OK;
  };
  ms_status st = MS_OK;
  if (nrun == 0) {
    st = energies_of(0);
  } else {
    std::vector<ms_status> res(nrun, MS_OK);
    std::vector<std::thread> threads;
    for (int r = 0; r < nrun; ++r) threads.emplace_back([&, r] { res[r] = energies_of(r); });
    for (auto& t : threads) t.join();
    for (int r = 0; r < nrun; ++r)
      if (res[r] != MS_OK && st == MS_OK) {
        st = res[r];
        ctx->last_error = run[r]->last_error;
      }
  }
  for (int r = 0; r < nrun; ++r) {   // join (also after an error)
    MS_HIP(ctx, hipEventRecord(ctx->sync_ev[1 + r], run[r]->stream));
    MS_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->sync_ev[1 + r], 0));
  }
  return st;
}

ms_status ms_star_cascade(ms_ctx ctx, const ms_smat* s, int64_t n_mats, ms_prec prec, ms_smat* whole) {
  if (!ctx) return MS_ERR_ARG;
  if (!s || n_mats <= 0) return fail(ctx, MS_ERR_ARG, "need at least one S-matrix");
  if (prec != MS_PREC_FP64 && prec != MS_PREC_FP32_MFMA) return fail(ctx, MS_ERR_ARG, "unknown precision");
  const int64_t n64 = s[0].n;
  if (n64 <= 0) return fail(ctx, MS_ERR_ARG, "s[0].n must be positive");
  if (n64 > MAX_N) return fail(ctx, MS_ERR_UNSUPPORTED, "n = %lld > %d", (long long)n64, MAX_N);
  for (int64_t i = 0; i < n_mats; ++i) MS_TRY(check_smat(ctx, s + i, n64, "s[i]"));
  MS_TRY(check_smat(ctx, whole, n64, "whole"));
  const void* wp[4] = {whole->t, whole->rp, whole->r, whole->tp};
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b)
      if (wp[a] == wp[b]) return fail(ctx, MS_ERR_ARG, "whole blocks must be distinct");
  for (int64_t i = 0; i < n_mats; ++i) {
    const void* sp[4] = {s[i].t, s[i].rp, s[i].r, s[i].tp};
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        if (wp[a] == sp[b]) return fail(ctx, MS_ERR_ARG, "whole aliases input %lld", (long long)i);
  }
  MS_HIP(ctx, hipSetDevice(ctx->device));
  const int n = (int)n64;
  const int64_t nn = (int64_t)n * n;
  const size_t bytes = nn * sizeof(double2);
  if (n_mats == 1) {
    MS_HIP(ctx, hipMemcpyAsync(whole->t, s[0].t, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    MS_HIP(ctx, hipMemcpyAsync(whole->rp, s[0].rp, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    MS_HIP(ctx, hipMemcpyAsync(whole->r, s[0].r, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    MS_HIP(ctx, hipMemcpyAsync(whole->tp, s[0].tp, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    return MS_OK;
  }
  void *acc0, *acc1;
  MS_TRY(workspace(ctx, WS_ACC0, 4 * bytes, &acc0));
  MS_TRY(workspace(ctx, WS_ACC1, 4 * bytes, &acc1));
  Blocks acc[2] = {{c2(acc0), c2(acc0) + nn, c2(acc0) + 2 * nn, c2(acc0) + 3 * nn},
                   {c2(acc1), c2(acc1) + nn, c2(acc1) + 2 * nn, c2(acc1) + 3 * nn}};
  Blocks a = blocks_of(s[0]);
  int cur = 0;
  for (int64_t i = 1; i < n_mats; ++i) {
    Blocks dst = (i == n_mats - 1) ? blocks_of(*whole) : acc[cur];
    MS_TRY(star(ctx, n, a, blocks_of(s[i]), dst, prec == MS_PREC_FP32_MFMA));
    a = dst;
    cur ^= 1;
  }
  return MS_OK;
}

// ------------------------------------------------------------------------------------------
ms_status ms_bloch_pencil(ms_ctx ctx, const ms_slices* cell, double energy, void* P, void* Q) {
  if (!ctx) return MS_ERR_ARG;
  MS_TRY(check_slices(ctx, cell));
  if (bad_ptr(cell->evec)) return fail(ctx, MS_ERR_ARG, "cell->evec (the slices' eigenvectors) is required");
  if (!std::isfinite(energy)) return fail(ctx, MS_ERR_ARG, "energy must be finite");
  if (bad_ptr(P) || bad_ptr(Q) || P == Q) return fail(ctx, MS_ERR_ARG, "P and Q must be distinct device buffers");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  const int n = (int)cell->n_g, m = (int)cell->n_slices;   // the cell's slices 1..m
  const int64_t nn = (int64_t)n * n;
  void *seg, *whole, *eps2, *ovl2;
  MS_TRY(workspace(ctx, WS_BSEG, (size_t)m * 4 * nn * sizeof(double2), &seg));
  MS_TRY(workspace(ctx, WS_BWHOLE, (size_t)4 * nn * sizeof(double2), &whole));
  std::vector<ms_smat> s(m);
  for (int i = 0; i < m; ++i) {
    double2* b = c2(seg) + (int64_t)i * 4 * nn;
    s[i] = ms_smat{n, b, b + nn, b + 2 * nn, b + 3 * nn};
  }
  // S(p, p+1) for p = 1..m-1 from the cell's own overlaps
  if (m > 1) MS_TRY(ms_slice_smatrix(ctx, cell, energy, 1, m, s.data()));
  // S(m, m+1): slice m joined to the next cell's slice 1 (thickness dz_1), through
  // O = U^m^dagger U^1 of the cell's own eigenvectors, so both Bloch planes share slice 1's
  // eigenbasis exactly; it is the interface 1|2 of a two-slice set (slice m, slice 1)
  MS_TRY(workspace(ctx, WS_BEPS, (size_t)(4 * n + 2) * sizeof(double), &eps2));
  MS_TRY(workspace(ctx, WS_BOVL, (size_t)3 * nn * sizeof(double2), &ovl2));
  double* e2 = (double*)eps2;
  const size_t row = n * sizeof(double);
  MS_HIP(ctx, hipMemcpyAsync(e2, cell->eps + (int64_t)m * n, row, hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(e2 + n, cell->eps + (int64_t)m * n, row, hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(e2 + 2 * n, cell->eps + n, row, hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(e2 + 3 * n, cell->eps + n, row, hipMemcpyDeviceToDevice, ctx->stream));
  double* dz2 = e2 + 4 * n;   // [dz_m, dz_1]
  MS_HIP(ctx, hipMemcpyAsync(dz2, cell->dz + (m - 1), sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(dz2 + 1, cell->dz, sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  const double2* U = c2(cell->evec);
  MS_TRY(gemm(ctx, n, n, n, U + (int64_t)(m - 1) * nn, n, OP_C, U, n, OP_N, c2(ovl2) + nn, n, ONE, ZERO));
  const ms_slices pair{n, 2, dz2, e2, ovl2, nullptr};
  MS_TRY(ms_slice_smatrix(ctx, &pair, energy, 1, 2, s.data() + (m - 1)));
  double2* w = c2(whole);
  ms_smat ws{n, w, w + nn, w + 2 * nn, w + 3 * nn};
  MS_TRY(ms_star_cascade(ctx, s.data(), m, MS_PREC_FP64, &ws));
  return launch_bloch_pencil(ctx, n, w, w + nn, w + 2 * nn, w + 3 * nn, static_cast<double2*>(P),
                             static_cast<double2*>(Q));
}

// ------------------------------------------------------------------------------------------
ms_status ms_transmission(ms_ctx ctx, const ms_smat* whole, double energy, const double* eps_left,
                          const double* eps_right, double* T, double* R, int64_t* n_open) {
  if (!ctx) return MS_ERR_ARG;
  if (!whole) return fail(ctx, MS_ERR_ARG, "whole is NULL");
  if (whole->n <= 0 || whole->n > MAX_N) return fail(ctx, MS_ERR_ARG, "bad whole.n");
  MS_TRY(check_smat(ctx, whole, whole->n, "whole"));
  if (bad_ptr(eps_left) || bad_ptr(eps_right) || bad_ptr(T) || bad_ptr(R) || bad_ptr(n_open))
    return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (!std::isfinite(energy)) return fail(ctx, MS_ERR_ARG, "energy must be finite");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  return launch_whole_T(ctx, (int)whole->n, energy, c2(whole->t), c2(whole->r), eps_left, eps_right, T, R, n_open,
                        ctx->d_status);
}

// ------------------------------------------------------------------------------------------
}  // extern "C"

namespace {

// The fused fold for n_k slice sets (equal sizes) and n_e energies each: instances
// i = k n_e + e, processed in sub-batches of consecutive instances.  Per interface the
// prologue, the LU and the back substitution run once over the whole sub-batch; the
// interface GEMM, the epilogue and the transmission columns run per slice set (each has
// its own overlaps and channel list) over its share of the sub-batch.
// ---- the fused right fold over several slice sets ------------------------------------------
//
// Every (slice set, energy) pair is one instance.  Sets are grouped by n_g; inside a group
// they are sorted by slice count, longest first, and each instance's k and P rows are stored
// right-aligned (slice p of a set with ns slices at row p + nsmax - ns), so at fold step s
// every set is at its interface p = ns - s, on the same rows, and the sets still folding are
// a prefix of the batch.  fold_plan does all host work (channel lists, uploads, workspace);
// fold_enqueue only launches kernels, so it can be captured into a graph.

struct FoldSet {            // one slice set and its energies [e0, e0 + ne) of the caller's arrays
  const ms_slices* sl;
  int64_t e0, ne;
};

struct FoldGroup {          // the sets of one n_g, longest first
  int n = 0, n_o = 0, n_oc = 1, nsmax = 0, nbi = 1;
  std::vector<int> sets;            // indices into FoldPlan::sets
  std::vector<int> n_ch;            // open channels of each set's right lead
  std::vector<int64_t> set_inst0;   // first instance of each set (fold order)
  int64_t inst0 = 0, ni = 0;        // the group's instances [inst0, inst0 + ni)
  int64_t ch0 = 0;                  // channel table [sets][n_oc] at ch0 of the channel buffer
  ms_ctx run = nullptr;             // context (stream, workspace) the group is enqueued on
  double cost = 0.0;                // n^3 x fold steps x instances, for placing groups on streams
  double2 *kb = nullptr, *pb = nullptr, *mm = nullptr, *yb = nullptr;
  void* aop = nullptr;
  int32_t *piv = nullptr, *sel = nullptr;
};

struct FoldPlan {
  std::vector<FoldSet> sets;
  std::vector<FoldGroup> groups;
  int64_t ni = 0;
  bool fp32 = false;
  const int32_t* ch = nullptr;     // device: channel tables
  const double* en = nullptr;      // device: energy of each instance (fold order)
  const int64_t* perm = nullptr;   // device: caller's index of each instance
  double* t = nullptr;             // device: results in fold order
  double* r = nullptr;
  int64_t* no = nullptr;
  int32_t* st = nullptr;
  int n_run = 0;                   // internal streams the groups are spread over (0: all on ctx)
};

struct FoldDims {
  int ldm, ldy;
  int64_t nn, sM, sY, sk;
  size_t asz, per_e;
};

FoldDims fold_dims(const FoldGroup& G, bool fp32) {
  FoldDims d;
  const int n = G.n;
  d.nn = (int64_t)n * n;
  d.ldm = 2 * n + G.n_o;
  d.ldy = n + G.n_o;
  d.sM = (int64_t)n * d.ldm;
  d.sY = (int64_t)n * d.ldy;
  d.sk = (int64_t)(G.nsmax + 2) * n;
  d.asz = fp32 ? sizeof(float2) : sizeof(double2);
  d.per_e = (size_t)(2 * d.sk) * sizeof(double2) + d.nn * d.asz + d.sM * sizeof(double2) +
            d.sY * sizeof(double2) + n * sizeof(int32_t);
  return d;
}

// the reusable fork/join events of the context (created outside any capture)
ms_status sync_events(ms_ctx ctx, size_t count) {
  while (ctx->sync_ev.size() < count) {
    hipEvent_t e = nullptr;
    MS_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->sync_ev.push_back(e);
  }
  return MS_OK;
}

ms_status fold_plan(ms_ctx ctx, const double* energies, ms_prec prec, FoldPlan& P) {
  MS_HIP(ctx, hipSetDevice(ctx->device));
  P.fp32 = prec == MS_PREC_FP32_MFMA;
  // groups by n_g in order of first appearance, longest set first inside a group
  for (int k = 0; k < (int)P.sets.size(); ++k) {
    if (P.sets[k].ne <= 0) continue;
    const int n = (int)P.sets[k].sl->n_g;
    auto it = std::find_if(P.groups.begin(), P.groups.end(), [&](const FoldGroup& g) { return g.n == n; });
    if (it == P.groups.end()) {
      P.groups.emplace_back();
      P.groups.back().n = n;
      it = P.groups.end() - 1;
    }
    it->sets.push_back(k);
  }
  std::vector<int32_t> chh;
  std::vector<double> enh;
  std::vector<int64_t> permh;
  std::vector<double> er;
  for (FoldGroup& G : P.groups) {
    std::stable_sort(G.sets.begin(), G.sets.end(),
                     [&](int a, int b) { return P.sets[a].sl->n_slices > P.sets[b].sl->n_slices; });
    G.nsmax = (int)P.sets[G.sets.front()].sl->n_slices;
    // open channels of each right lead at that set's highest energy, lowest first; the
    // tables are padded to the longest with -1 (columns that stay zero)
    std::vector<std::vector<int32_t>> chs(G.sets.size());
    er.resize(G.n);
    for (size_t j = 0; j < G.sets.size(); ++j) {
      const FoldSet& fs = P.sets[G.sets[j]];
      const double* eps_r = fs.sl->eps + (int64_t)(fs.sl->n_slices + 1) * G.n;
      MS_HIP(ctx, hipMemcpyAsync(er.data(), eps_r, G.n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      MS_HIP(ctx, hipStreamSynchronize(ctx->stream));
      const double emax = *std::max_element(energies + fs.e0, energies + fs.e0 + fs.ne);
      for (int i = 0; i < G.n; ++i)
        if (er[i] < emax) chs[j].push_back(i);
      std::stable_sort(chs[j].begin(), chs[j].end(), [&](int32_t x, int32_t y) { return er[x] < er[y]; });
      G.n_o = std::max(G.n_o, (int)chs[j].size());
    }
    G.n_oc = std::max(1, G.n_o);
    G.ch0 = (int64_t)chh.size();
    G.inst0 = P.ni;
    for (size_t j = 0; j < G.sets.size(); ++j) {
      const FoldSet& fs = P.sets[G.sets[j]];
      G.n_ch.push_back((int)chs[j].size());
      std::vector<int32_t> row(G.n_oc, -1);
      std::copy(chs[j].begin(), chs[j].end(), row.begin());
      chh.insert(chh.end(), row.begin(), row.end());
      G.set_inst0.push_back(P.ni);
      for (int64_t e = 0; e < fs.ne; ++e) {
        enh.push_back(energies[fs.e0 + e]);
        permh.push_back(fs.e0 + e);
      }
      P.ni += fs.ne;
    }
    G.ni = P.ni - G.inst0;
    for (int k : G.sets) G.cost += (double)G.n * G.n * G.n * (P.sets[k].sl->n_slices + 1) * P.sets[k].ne;
  }
  if (P.ni == 0) return MS_OK;
  // Groups of different n_g are independent: with several, they are spread over up to
  // three internal contexts (own stream and workspace), heaviest first onto the least
  // loaded, and run concurrently (MS_FOLD_GROUP_STREAMS=0 keeps them on the caller's stream).
  {
    bool spread = P.groups.size() > 1;
    if (const char* env = getenv("MS_FOLD_GROUP_STREAMS")) spread = spread && atoi(env) != 0;
    P.n_run = spread ? (int)std::min<size_t>(3, P.groups.size()) : 0;
    std::vector<int> order(P.groups.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return P.groups[a].cost > P.groups[b].cost; });
    std::vector<double> load(std::max(1, P.n_run), 0.0);
    for (int gi : order) {
      FoldGroup& G = P.groups[gi];
      if (P.n_run == 0) {
        G.run = ctx;
        continue;
      }
      const int r = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[r] += G.cost;
      MS_TRY(child(ctx, r, &G.run));
      G.run->tiles = ctx->tiles;
      G.run->use_gws = ctx->use_gws;
    }
    if (P.n_run > 0) MS_TRY(sync_events(ctx, 1 + P.n_run));
  }
  // each group's scratch comes from its runner's workspace; a runner that serves several
  // groups (one after the other on its stream) is first grown to the largest need per slot,
  // so no later request moves a buffer an earlier group already holds
  const int slots[7] = {WS_K, WS_P, WS_AOP, WS_M, WS_Y, WS_PIV, WS_SEL};
  // allocation-free mode (one group): the arena left for the per-instance scratch
  const size_t arena_left =
      ctx->arena ? ctx->arena_size - std::min(ctx->arena_size, ctx->arena_used + ARENA_TABLES) : 0;
  if (ctx->arena && P.groups.size() != 1)
    return fail(ctx, MS_ERR_UNSUPPORTED, "the allocation-free fold takes slice sets of one basis size");
  auto needs = [&](FoldGroup& G, size_t* nd) {
    const FoldDims d = fold_dims(G, P.fp32);
    // sub-batch: the instances whose scratch fits the budget (in the allocation-free mode what
    // is left of the arena after the tables, the LU's workspace counted per instance)
    int64_t fit = (int64_t)(BATCH_BUDGET / d.per_e);
    if (ctx->arena) fit = (int64_t)(arena_left / (d.per_e + lu_bytes_per_matrix(G.n, d.ldm) + 10 * 256));
    const int64_t nbi = std::max<int64_t>(1, std::min<int64_t>(G.ni, fit));
    G.nbi = (int)std::min<int64_t>(nbi, 65535);
    nd[0] = nd[1] = (size_t)G.nbi * d.sk * sizeof(double2);
    nd[2] = (size_t)G.nbi * d.nn * d.asz;
    nd[3] = (size_t)G.nbi * d.sM * sizeof(double2);
    nd[4] = (size_t)G.nbi * d.sY * sizeof(double2);
    nd[5] = (size_t)G.nbi * G.n * sizeof(int32_t);
    nd[6] = (size_t)G.nbi * (THRESH_CAP + 1) * sizeof(int32_t);
    return d;
  };
  for (FoldGroup& G : P.groups) {   // pass 1: grow every runner to its groups' largest needs
    size_t nd[7];
    const FoldDims d = needs(G, nd);
    void* v;
    for (int i = 0; i < 7; ++i) {
      size_t most = nd[i];
      for (FoldGroup& H : P.groups)
        if (H.run == G.run) {
          size_t nh[7];
          needs(H, nh);
          most = std::max(most, nh[i]);
        }
      MS_TRY(workspace(G.run, slots[i], most, &v));
    }
    MS_TRY(lu_reserve(G.run, G.n, d.ldm, G.nbi));
  }
  for (FoldGroup& G : P.groups) {   // pass 2: take the pointers (no slot grows any more)
    ms_ctx c = G.run;
    void* v;
    MS_TRY(workspace(c, WS_K, 1, &v));
    G.kb = c2(v);
    MS_TRY(workspace(c, WS_P, 1, &v));
    G.pb = c2(v);
    MS_TRY(workspace(c, WS_AOP, 1, &G.aop));
    MS_TRY(workspace(c, WS_M, 1, &v));
    G.mm = c2(v);
    MS_TRY(workspace(c, WS_Y, 1, &v));
    G.yb = c2(v);
    MS_TRY(workspace(c, WS_PIV, 1, &v));
    G.piv = (int32_t*)v;
    MS_TRY(workspace(c, WS_SEL, 1, &v));
    G.sel = (int32_t*)v;
  }
  void *chd, *end, *pmd, *v;
  MS_TRY(workspace(ctx, WS_CH, chh.size() * sizeof(int32_t), &chd));
  MS_TRY(upload(ctx, chd, chh.data(), chh.size() * sizeof(int32_t)));
  MS_TRY(workspace(ctx, WS_EN, P.ni * sizeof(double), &end));
  MS_TRY(upload(ctx, end, enh.data(), P.ni * sizeof(double)));
  MS_TRY(workspace(ctx, WS_PERM, P.ni * sizeof(int64_t), &pmd));
  MS_TRY(upload(ctx, pmd, permh.data(), P.ni * sizeof(int64_t)));
  P.ch = (const int32_t*)chd;
  P.en = (const double*)end;
  P.perm = (const int64_t*)pmd;
  MS_TRY(workspace(ctx, WS_RT, P.ni * sizeof(double), &v));
  P.t = (double*)v;
  MS_TRY(workspace(ctx, WS_RR, P.ni * sizeof(double), &v));
  P.r = (double*)v;
  MS_TRY(workspace(ctx, WS_RNO, P.ni * sizeof(int64_t), &v));
  P.no = (int64_t*)v;
  MS_TRY(workspace(ctx, WS_RST, P.ni * sizeof(int32_t), &v));
  P.st = (int32_t*)v;
  return MS_OK;
}

// the kernels of one group, on its runner's stream
ms_status enqueue_group(ms_ctx c, const FoldPlan& P, const FoldGroup& G) {
  const bool fp32 = P.fp32;
  const int n = G.n, n_o = G.n_o;
  const FoldDims d = fold_dims(G, fp32);
  const int64_t nn = d.nn, sk = d.sk, sM = d.sM, sY = d.sY;
  for (int64_t i0 = 0; i0 < G.ni; i0 += G.nbi) {
    const int be = (int)std::min<int64_t>(G.nbi, G.ni - i0);
    const int64_t g0 = G.inst0 + i0;   // fold-order index of local instance 0
    struct Seg { int j, a, m, ns; };   // group set j owns local instances [a, a + m)
    std::vector<Seg> segs;
    for (int j = 0; j < (int)G.sets.size(); ++j) {
      const int64_t s0 = G.set_inst0[j] - G.inst0, s1 = s0 + P.sets[G.sets[j]].ne;
      const int64_t lo = std::max<int64_t>(i0, s0), hi = std::min<int64_t>(i0 + be, s1);
      if (lo < hi) segs.push_back(Seg{j, (int)(lo - i0), (int)(hi - lo), (int)P.sets[G.sets[j]].sl->n_slices});
    }
    for (const Seg& g : segs) {
      const ms_slices* sl = P.sets[G.sets[g.j]].sl;
      const int64_t off = (int64_t)g.a * sk + (int64_t)(G.nsmax - g.ns) * n;
      MS_TRY(launch_wavevectors(c, n, g.ns + 2, g.m, sl->eps, P.en + g0 + g.a, sl->dz, G.kb + off, G.pb + off, sk));
    }
    const int smax = segs.front().ns;   // the longest set of the sub-batch comes first
    for (int s = 0; s <= smax; ++s) {
      int act = 0;                      // instances still folding: a prefix of the sub-batch
      for (const Seg& g : segs)
        if (g.ns >= s) act = g.a + g.m;
      const int64_t q = G.nsmax - s;    // row of slice p = ns - s in every set
      const double2* kp = G.kb + q * n;
      const double2* kq = G.kb + (q + 1) * n;
      const double2* pq = G.pb + (q + 1) * n;
      const bool first = (s == 0);
      if (!first) {
        if (fp32) MS_TRY(launch_thresh_select(c, n, act, kq, sk, THRESH_K, THRESH_CAP, G.sel));
        MS_TRY(launch_prologue(c, n, act, G.yb, d.ldy, sY, kq, pq, sk, fp32 ? G.sel : nullptr, THRESH_CAP, G.aop,
                               fp32));
        for (const Seg& g : segs) {
          if (g.ns < s) break;
          // W = rho^T [C- | C+ off its diagonal] for the set's energies, B generated from the
          // set's O (shared by its energies) and each energy's k of slices p and p+1
          const double2* O = c2(P.sets[G.sets[g.j]].sl->ovl) + (int64_t)(g.ns - s) * nn;
          GemmArgs gm;
          gm.M = n; gm.N = 2 * n; gm.K = n;
          gm.A = static_cast<char*>(G.aop) + (size_t)g.a * nn * d.asz; gm.lda = n; gm.sA = nn; gm.opA = OP_N;
          gm.B = O; gm.ldb = n; gm.sB = 0; gm.opB = OP_T;
          // the product's epilogue writes [Phi_A^T | Phi_B^T] straight into the augmented matrix
          gm.C = G.mm + g.a * sM; gm.ldc = d.ldm; gm.sC = sM;
          gm.batch = g.m;
          gm.kp = kp + g.a * sk; gm.kq = kq + g.a * sk; gm.sk = sk;
          gm.ey = G.yb + g.a * sY; gm.eldy = d.ldy; gm.esy = sY;
          gm.epq = pq + g.a * sk;
          gm.esel = fp32 ? G.sel + (int64_t)g.a * (THRESH_CAP + 1) : nullptr;
          gm.ecap = THRESH_CAP;
          gm.prof = PC_IFACE_GEMM;
          MS_TRY(fp32 ? cgemm32(c, gm) : zgemm(c, gm));
        }
      }
      for (const Seg& g : segs) {
        if (g.ns < s) break;
        if (first) {   // no product at the first interface: C+- alone
          const double2* O = c2(P.sets[G.sets[g.j]].sl->ovl) + (int64_t)(g.ns - s) * nn;
          MS_TRY(launch_epilogue(c, n, g.m, O, nullptr, kp + g.a * sk, kq + g.a * sk, pq + g.a * sk, sk,
                                 G.yb + g.a * sY, d.ldy, sY, nullptr, THRESH_CAP, G.mm + g.a * sM, d.ldm, sM));
        }
        MS_TRY(launch_tcols(c, n, n_o, g.m, P.ch + G.ch0 + (int64_t)g.j * G.n_oc, G.yb + g.a * sY, d.ldy, sY, n,
                            kq + g.a * sk, pq + g.a * sk, sk, first ? 1 : 0, G.mm + g.a * sM, d.ldm, sM));
      }
      MS_TRY(getrf_aug(c, G.mm, n, d.ldm, sM, act, G.piv, P.st + g0, 1));
      MS_TRY(trsm_upper_aug(c, G.mm, n, d.ldm, sM, act, G.yb, d.ldy, sY, P.st + g0, 1));
    }
    for (const Seg& g : segs) {
      const ms_slices* sl = P.sets[G.sets[g.j]].sl;
      const double* eps_l = sl->eps;
      const double* eps_r = sl->eps + (int64_t)(g.ns + 1) * n;
      const int64_t o = g0 + g.a;
      MS_TRY(launch_batch_T(c, n, G.n_ch[g.j], g.m, P.ch + G.ch0 + (int64_t)g.j * G.n_oc, P.en + o, eps_l, eps_r,
                            G.yb + g.a * sY, d.ldy, sY, P.t + o, P.r + o, P.no + o, P.st + o));
    }
  }
  return MS_OK;
}

ms_status fold_enqueue(ms_ctx ctx, const FoldPlan& P, double* T, double* R, int64_t* n_open, int32_t* status) {
  if (P.ni == 0) return MS_OK;
  MS_TRY(launch_fill_i32(ctx, P.ni, P.st, 0));
  std::vector<ms_ctx> runners;   // internal contexts in use, each forked from and joined to ctx
  for (const FoldGroup& G : P.groups)
    if (G.run != ctx && std::find(runners.begin(), runners.end(), G.run) == runners.end()) runners.push_back(G.run);
  if (!runners.empty()) {
    MS_HIP(ctx, hipEventRecord(ctx->sync_ev[0], ctx->stream));
    for (ms_ctx c : runners) MS_HIP(ctx, hipStreamWaitEvent(c->stream, ctx->sync_ev[0], 0));
  }
  ms_status s = MS_OK;
  for (const FoldGroup& G : P.groups) {
    ms_ctx c = G.run;
    c->tile_n = G.n;   // GEMM tiles of the group's basis size
    if (c != ctx) {   // the runner counts against what is left of the graph's budget
      c->capturing = ctx->capturing;
      c->cap_limit = ctx->cap_limit - ctx->cap_kernels;
      c->cap_kernels = 0;
    }
    s = enqueue_group(c, P, G);
    c->tile_n = 0;
    if (c != ctx) {
      c->capturing = false;
      ctx->cap_kernels += c->cap_kernels;
      if (s == MS_OK && ctx->capturing && ctx->cap_kernels > ctx->cap_limit)
        s = fail(ctx, MS_ERR_UNSUPPORTED,
                 "the fold needs more than %lld kernels in one graph; split the sets over several calls "
                 "or call without MS_FOLD_GRAPH", (long long)ctx->cap_limit);
      if (s != MS_OK && !c->last_error.empty()) ctx->last_error = c->last_error;
    }
    if (s != MS_OK) break;
  }
  // join every runner back into the caller's stream (also after an error, so a capture
  // can be ended), after all groups have been enqueued
  for (size_t i = 0; i < runners.size(); ++i) {
    MS_HIP(ctx, hipEventRecord(ctx->sync_ev[1 + i], runners[i]->stream));
    MS_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->sync_ev[1 + i], 0));
  }
  MS_TRY(s);
  return launch_scatter_results(ctx, P.ni, P.perm, P.t, P.r, P.no, P.st, T, R, n_open, status);
}

// plan + enqueue; with `graph` the plan's tables and every scratch buffer come from the
// graph's own workspace and the enqueue is captured (on the context's capture stream) into
// one hipGraph, which is launched on the context's stream and kept for ms_graph_replay
ms_status fold_run(ms_ctx ctx, FoldPlan& P, const double* energies, ms_prec prec, bool graph, double* T, double* R,
                   int64_t* n_open, int32_t* point_status) {
  if (!graph) {
    MS_TRY(fold_plan(ctx, energies, prec, P));
    return fold_enqueue(ctx, P, T, R, n_open, point_status);
  }
  if (ctx->graph) {   // its workspace is about to be reused
    MS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    MS_HIP(ctx, hipGraphExecDestroy(ctx->graph));
    ctx->graph = nullptr;
  }
  if (!ctx->cap_stream) MS_HIP(ctx, hipStreamCreate(&ctx->cap_stream));
  ctx->use_gws = true;
  ms_status s = fold_plan(ctx, energies, prec, P);
  if (s != MS_OK) {
    ctx->use_gws = false;
    for (ms_ctx k : ctx->kids) k->use_gws = false;
    return s;
  }
  const hipStream_t main = ctx->stream;
  // Graphs of up to about 93k kernels (folds of N_G 200-800 with up to 390 slices) have been
  // captured, instantiated and replayed; a capture of 213k kernels ended the process during
  // the capture or instantiation, so one capture holds at most MAX_GRAPH_KERNELS (less if
  // MS_GRAPH_MAX_KERNELS says so).
  ctx->cap_limit = MAX_GRAPH_KERNELS;
  if (const char* env = getenv("MS_GRAPH_MAX_KERNELS"))
    ctx->cap_limit = std::max<int64_t>(1, std::min<int64_t>(MAX_GRAPH_KERNELS, atoll(env)));
  ctx->cap_kernels = 0;
  const hipError_t eb = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
  if (eb != hipSuccess) {
    ctx->use_gws = false;
    for (ms_ctx k : ctx->kids) k->use_gws = false;
    return hip_fail(ctx, eb, "hipStreamBeginCapture");
  }
  ctx->stream = ctx->cap_stream;
  ctx->capturing = true;
  s = fold_enqueue(ctx, P, T, R, n_open, point_status);
  ctx->capturing = false;
  ctx->use_gws = false;
  for (ms_ctx k : ctx->kids) k->use_gws = false;
  ctx->stream = main;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
  if (s != MS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
  hipGraphExec_t x = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return hip_fail(ctx, e2, "hipGraphInstantiate");
  ctx->graph = x;
  MS_HIP(ctx, hipGraphLaunch(x, ctx->stream));
  return MS_OK;
}

ms_status check_energies(ms_ctx ctx, int64_t count, const double* energies) {
  for (int64_t e = 0; e < count; ++e)
    if (!std::isfinite(energies[e])) return fail(ctx, MS_ERR_ARG, "energy %lld is not finite", (long long)e);
  return MS_OK;
}

}  // namespace

extern "C" {

ms_status ms_transmission_batch(ms_ctx ctx, const ms_slices* slices, int64_t n_e, const double* energies,
                                ms_prec prec, double* T, double* R, int64_t* n_open, int32_t* point_status) {
  if (!ctx) return MS_ERR_ARG;
  MS_TRY(check_slices(ctx, slices));
  if (n_e < 0) return fail(ctx, MS_ERR_ARG, "n_e must be >= 0");
  if (n_e == 0) return MS_OK;
  if (bad_ptr(energies) || bad_ptr(T) || bad_ptr(R) || bad_ptr(n_open) || bad_ptr(point_status))
    return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (prec != MS_PREC_FP64 && prec != MS_PREC_FP32_MFMA) return fail(ctx, MS_ERR_ARG, "unknown precision");
  MS_TRY(check_energies(ctx, n_e, energies));
  FoldPlan P;
  P.sets.push_back(FoldSet{slices, 0, n_e});
  return fold_run(ctx, P, energies, prec, false, T, R, n_open, point_status);
}

ms_status ms_transmission_multi(ms_ctx ctx, int64_t n_k, const ms_slices* slices, int64_t n_e,
                                const double* energies, ms_prec prec, double* T, double* R, int64_t* n_open,
                                int32_t* point_status) {
  if (!ctx) return MS_ERR_ARG;
  if (n_k < 0 || n_e < 0) return fail(ctx, MS_ERR_ARG, "n_k and n_e must be >= 0");
  if (n_k == 0 || n_e == 0) return MS_OK;
  if (bad_ptr(slices) || bad_ptr(energies) || bad_ptr(T) || bad_ptr(R) || bad_ptr(n_open) || bad_ptr(point_status))
    return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (n_k > 65535) return fail(ctx, MS_ERR_UNSUPPORTED, "n_k %lld > 65535", (long long)n_k);
  for (int64_t k = 0; k < n_k; ++k) {
    MS_TRY(check_slices(ctx, slices + k));
    if (slices[k].n_g != slices[0].n_g || slices[k].n_slices != slices[0].n_slices)
      return fail(ctx, MS_ERR_ARG, "slice set %lld has other sizes than set 0", (long long)k);
  }
  if (prec != MS_PREC_FP64 && prec != MS_PREC_FP32_MFMA) return fail(ctx, MS_ERR_ARG, "unknown precision");
  MS_TRY(check_energies(ctx, n_k * n_e, energies));
  FoldPlan P;
  for (int64_t k = 0; k < n_k; ++k) P.sets.push_back(FoldSet{slices + k, k * n_e, n_e});
  return fold_run(ctx, P, energies, prec, false, T, R, n_open, point_status);
}

ms_status ms_transmission_uneven(ms_ctx ctx, int64_t n_sets, const ms_slices* sets, const int64_t* n_e,
                                 const double* energies, ms_prec prec, int32_t flags, double* T, double* R,
                                 int64_t* n_open, int32_t* point_status) {
  if (!ctx) return MS_ERR_ARG;
  if (n_sets < 0) return fail(ctx, MS_ERR_ARG, "n_sets must be >= 0");
  if (n_sets == 0) return MS_OK;
  if (bad_ptr(sets) || bad_ptr(n_e)) return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (flags & ~(int32_t)MS_FOLD_GRAPH) return fail(ctx, MS_ERR_ARG, "unknown flags 0x%x", (unsigned)flags);
  if (prec != MS_PREC_FP64 && prec != MS_PREC_FP32_MFMA) return fail(ctx, MS_ERR_ARG, "unknown precision");
  FoldPlan P;
  int64_t total = 0;
  for (int64_t k = 0; k < n_sets; ++k) {
    MS_TRY(check_slices(ctx, sets + k));
    if (n_e[k] < 0) return fail(ctx, MS_ERR_ARG, "n_e[%lld] < 0", (long long)k);
    P.sets.push_back(FoldSet{sets + k, total, n_e[k]});
    total += n_e[k];
  }
  if (total == 0) return MS_OK;
  if (bad_ptr(energies) || bad_ptr(T) || bad_ptr(R) || bad_ptr(n_open) || bad_ptr(point_status))
    return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  MS_TRY(check_energies(ctx, total, energies));
  return fold_run(ctx, P, energies, prec, (flags & MS_FOLD_GRAPH) != 0, T, R, n_open, point_status);
}

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// the device address of `scratch` on ctx's device (looked up once per device, with that
// device current)
ms_status scratch_of(ms_ctx ctx, char** out) {
  if (ctx->device < 0 || ctx->device >= MAX_DEVICES)
    return fail(ctx, MS_ERR_UNSUPPORTED, "device %d beyond the %d the scratch table holds", ctx->device, MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[ctx->device] = p;
  }
  *out = static_cast<char*>(g_scratch_ptr[ctx->device]);
  return MS_OK;
}
}  // namespace

ms_status ms_transmission_batch_noalloc(ms_ctx ctx, const ms_slices* slices, int64_t n_e, const double* energies,
                                        ms_prec prec, double* T, double* R, int64_t* n_open, int32_t* point_status) {
  if (!ctx) return MS_ERR_ARG;
  MS_TRY(check_slices(ctx, slices));
  if (n_e < 0) return fail(ctx, MS_ERR_ARG, "n_e must be >= 0");
  if (n_e == 0) return MS_OK;
  if (bad_ptr(energies) || bad_ptr(T) || bad_ptr(R) || bad_ptr(n_open) || bad_ptr(point_status))
    return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  if (prec != MS_PREC_FP64 && prec != MS_PREC_FP32_MFMA) return fail(ctx, MS_ERR_ARG, "unknown precision");
  MS_TRY(check_energies(ctx, n_e, energies));
  if (ctx->capturing) return fail(ctx, MS_ERR_UNSUPPORTED, "called inside the library's own capture");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  char* base = nullptr;
  MS_TRY(scratch_of(ctx, &base));
  // every call carves its slots from the start of the device's scratch
  ctx->arena = base;
  ctx->arena_size = MS_NOALLOC_SCRATCH_BYTES;
  ctx->arena_used = 0;
  ctx->aws.clear();
  ctx->aws_size.clear();
  FoldPlan P;
  P.sets.push_back(FoldSet{slices, 0, n_e});
  const ms_status st = fold_run(ctx, P, energies, prec, false, T, R, n_open, point_status);
  ctx->arena = nullptr;
  ctx->arena_size = ctx->arena_used = 0;
  ctx->aws.clear();
  ctx->aws_size.clear();
  return st;
}

ms_status ms_graph_replay(ms_ctx ctx) {
  if (!ctx) return MS_ERR_ARG;
  if (!ctx->graph) return fail(ctx, MS_ERR_ARG, "no captured graph on this context");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  MS_HIP(ctx, hipGraphLaunch(ctx->graph, ctx->stream));
  return MS_OK;
}

// ------------------------------------------------------------------------------------------
// Doubling with the mixed recurrence (App. A, Eq. recurrence2), then the star product.
namespace {

struct BlockSet {   // four arrays of n x n blocks: (I11, I12, S21, S22) or (S11, S12, S21, S22)
  double2 *a11, *a12, *r, *tp;
};

ms_status mm(ms_ctx ctx, int n, const double2* A, int64_t lda, int64_t sA, const double2* B, int64_t ldb, int64_t sB,
             double2* C, int64_t ldc, int64_t sC, int batch, double alpha, double beta) {
  GemmArgs g;
  g.M = n; g.N = n; g.K = n;
  g.A = A; g.lda = lda; g.sA = sA;
  g.B = B; g.ldb = ldb; g.sB = sB;
  g.C = C; g.ldc = ldc; g.sC = sC;
  g.batch = batch;
  g.alpha = make_double2(alpha, 0.0);
  g.beta = make_double2(beta, 0.0);
  return zgemm(ctx, g);
}

}  // namespace

ms_status ms_mixed_doubling(ms_ctx ctx, const ms_slices* slices, double energy, double max_cond, ms_smat* whole,
                            int32_t* mixed_levels) {
  if (!ctx) return MS_ERR_ARG;
  MS_TRY(check_slices(ctx, slices));
  if (!std::isfinite(energy)) return fail(ctx, MS_ERR_ARG, "energy must be finite");
  if (!(max_cond >= 1.0)) return fail(ctx, MS_ERR_ARG, "max_cond must be >= 1 (may be +inf)");
  if (!mixed_levels) return fail(ctx, MS_ERR_ARG, "mixed_levels is NULL");
  MS_TRY(check_smat(ctx, whole, slices->n_g, "whole"));
  {
    const void* wp[4] = {whole->t, whole->rp, whole->r, whole->tp};
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        if (wp[a] == wp[b]) return fail(ctx, MS_ERR_ARG, "whole blocks must be distinct");
  }
  MS_HIP(ctx, hipSetDevice(ctx->device));
  const int n = (int)slices->n_g, ns = (int)slices->n_slices, nrows = ns + 2;
  const int64_t nn = (int64_t)n * n;
  const int nb0 = ns + 1;                 // interfaces S(p,p+1), p = 0..ns
  const int half = nb0 / 2 + 1;           // the most blocks any later level holds
  void *en, *kb, *pb, *sa, *sb, *aug, *inv, *tmp, *piv, *nrm;
  MS_TRY(workspace(ctx, WS_EN, sizeof(double), &en));
  MS_TRY(upload(ctx, en, &energy, sizeof(double)));
  MS_TRY(workspace(ctx, WS_K, (size_t)nrows * n * sizeof(double2), &kb));
  MS_TRY(workspace(ctx, WS_P, (size_t)nrows * n * sizeof(double2), &pb));
  MS_TRY(launch_wavevectors(ctx, n, nrows, 1, slices->eps, (const double*)en, slices->dz, c2(kb), c2(pb)));
  MS_TRY(workspace(ctx, WS_MD_A, (size_t)4 * nb0 * nn * sizeof(double2), &sa));
  MS_TRY(workspace(ctx, WS_MD_B, (size_t)4 * half * nn * sizeof(double2), &sb));
  MS_TRY(workspace(ctx, WS_AUG, (size_t)half * 3 * nn * sizeof(double2), &aug));
  MS_TRY(workspace(ctx, WS_MD_INV, (size_t)half * nn * sizeof(double2), &inv));
  MS_TRY(workspace(ctx, WS_MD_T, (size_t)5 * half * nn * sizeof(double2), &tmp));
  MS_TRY(workspace(ctx, WS_PIV, (size_t)half * n * sizeof(int32_t), &piv));
  MS_TRY(workspace(ctx, WS_MD_NRM, (size_t)2 * nb0 * sizeof(double), &nrm));
  BlockSet A{c2(sa), c2(sa) + (int64_t)nb0 * nn, c2(sa) + 2 * (int64_t)nb0 * nn, c2(sa) + 3 * (int64_t)nb0 * nn};
  BlockSet B{c2(sb), c2(sb) + (int64_t)half * nn, c2(sb) + 2 * (int64_t)half * nn, c2(sb) + 3 * (int64_t)half * nn};
  double2* AUG = c2(aug);
  double2* INV = c2(inv);
  double2* T0 = c2(tmp);
  int32_t* PIV = (int32_t*)piv;
  double* NRM = (double*)nrm;
  const double2* ovl = c2(slices->ovl);

  // level 0: S21, S22 in the cancelled form of Eq. scatter, I11 = X P^-1, I12 = Y P (Eq. transfer)
  for (int q = 0; q < nb0; q += half) {
    const int bc = std::min(half, nb0 - q);
    double2 *xc = T0, *yc = T0 + (int64_t)bc * nn, *z = T0 + 2 * (int64_t)bc * nn;
    MS_TRY(launch_xy(ctx, n, bc, ovl, c2(kb), q, AUG, xc, yc));   // [X | I | Y]
    MS_TRY(getrf_aug(ctx, AUG, n, 3 * n, 3 * nn, bc, PIV, ctx->d_status, 0));
    MS_TRY(trsm_upper_aug(ctx, AUG, n, 3 * n, 3 * nn, bc, z, 2 * n, 2 * nn, ctx->d_status, 0));
    MS_TRY(mm(ctx, n, yc, n, nn, z, 2 * n, 2 * nn, A.r + q * nn, n, nn, bc, 1.0, 0.0));        // Y X^-1
    MS_TRY(mm(ctx, n, yc, n, nn, z + n, 2 * n, 2 * nn, xc, n, nn, bc, -1.0, 1.0));            // X - Y X^-1 Y
    MS_TRY(launch_smat_finish(ctx, n, bc, z, xc, c2(pb), q, A.a11 + q * nn, A.a12 + q * nn, A.tp + q * nn));
    MS_TRY(launch_transfer_blocks(ctx, n, bc, ovl, c2(kb), c2(pb), q, A.a11 + q * nn, A.a12 + q * nn));
  }

  // max_i cond_1(I11_i) over the nb blocks of S; with `convert`, also S11 = I11^-1 and
  // S12 = -I11^-1 I12 in place (Eq. scatter)
  auto cond_pass = [&](BlockSet& S, int nb, bool convert, double* cmax) -> ms_status {
    for (int q = 0; q < nb; q += half) {
      const int bc = std::min(half, nb - q);
      MS_TRY(launch_aug_build(ctx, n, bc, 2 * n, S.a11 + q * nn, nn, nullptr, 0, nullptr, 0, AUG));
      MS_TRY(getrf_aug(ctx, AUG, n, 2 * n, 2 * nn, bc, PIV, ctx->d_status, 0));
      MS_TRY(trsm_upper_aug(ctx, AUG, n, 2 * n, 2 * nn, bc, INV, n, nn, ctx->d_status, 0));
      if (convert) {
        MS_TRY(mm(ctx, n, INV, n, nn, S.a12 + q * nn, n, nn, T0, n, nn, bc, -1.0, 0.0));
        MS_TRY(launch_axpby(ctx, nn, bc, 1.0, T0, nn, 0.0, nullptr, 0, S.a12 + q * nn, nn));
        MS_TRY(launch_axpby(ctx, nn, bc, 1.0, INV, nn, 0.0, nullptr, 0, S.a11 + q * nn, nn));
      } else {
        MS_TRY(launch_norm1(ctx, n, bc, S.a11 + q * nn, n, nn, NRM + q));
        MS_TRY(launch_norm1(ctx, n, bc, INV, n, nn, NRM + nb0 + q));
      }
    }
    if (!convert) {
      std::vector<double> h(2 * (size_t)nb0);
      MS_HIP(ctx, hipMemcpyAsync(h.data(), NRM, h.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      MS_HIP(ctx, hipStreamSynchronize(ctx->stream));
      double c = 0.0;
      for (int i = 0; i < nb; ++i) {
        const double v = h[i] * h[nb0 + i];
        c = (v == v) ? std::max(c, v) : INFINITY;
      }
      *cmax = c;
    }
    return MS_OK;
  };

  BlockSet* cur = &A;
  BlockSet* nxt = &B;
  int nb = nb0, levels = 0;
  double cmax = 0.0;
  MS_TRY(cond_pass(*cur, nb, false, &cmax));
  bool mixed = cmax <= max_cond;
  if (!mixed) MS_TRY(cond_pass(*cur, nb, true, nullptr));
  while (nb > 1) {
    const int np = nb / 2;
    const int64_t s2 = 2 * nn;
    BlockSet& X = *cur;
    BlockSet& Y = *nxt;
    if (mixed) {   // Eq. recurrence2: a = block 2i, b = block 2i+1
      double2 *W = T0, *Q = T0 + (int64_t)np * nn, *QM = T0 + 2 * (int64_t)np * nn;
      MS_TRY(launch_aug_build(ctx, n, np, 2 * n, X.a11, s2, nullptr, 0, nullptr, 0, AUG));       // [I11_a | I]
      MS_TRY(mm(ctx, n, X.a12, n, s2, X.r + nn, n, s2, AUG, 2 * n, s2, np, 1.0, 1.0));          // M
      MS_TRY(mm(ctx, n, X.a12, n, s2, X.tp + nn, n, s2, W, n, nn, np, 1.0, 0.0));               // W = I12_a S22_b
      MS_TRY(launch_axpby(ctx, nn, np, 1.0, W, nn, 0.0, nullptr, 0, Y.a12, nn));
      MS_TRY(mm(ctx, n, AUG, 2 * n, s2, X.a12 + nn, n, s2, Y.a12, n, nn, np, 1.0, 1.0));       // I12 = M I12_b + W
      MS_TRY(mm(ctx, n, AUG, 2 * n, s2, X.a11 + nn, n, s2, Y.a11, n, nn, np, 1.0, 0.0));       // I11 = M I11_b
      MS_TRY(getrf_aug(ctx, AUG, n, 2 * n, s2, np, PIV, ctx->d_status, 0));
      MS_TRY(trsm_upper_aug(ctx, AUG, n, 2 * n, s2, np, INV, n, nn, ctx->d_status, 0));         // M^-1
      MS_TRY(mm(ctx, n, X.tp, n, s2, X.r + nn, n, s2, Q, n, nn, np, 1.0, 0.0));                 // S22_a S21_b
      MS_TRY(mm(ctx, n, Q, n, nn, INV, n, nn, QM, n, nn, np, 1.0, 0.0));                        // ... M^-1
      MS_TRY(launch_axpby(ctx, nn, np, 1.0, X.r, s2, 1.0, QM, nn, Y.r, nn));                    // S21
      MS_TRY(mm(ctx, n, X.tp, n, s2, X.tp + nn, n, s2, Y.tp, n, nn, np, 1.0, 0.0));
      MS_TRY(mm(ctx, n, QM, n, nn, W, n, nn, Y.tp, n, nn, np, -1.0, 1.0));                      // S22
    } else {       // Eq. recurrence: the star product of a = block 2i and b = block 2i+1
      double2 *Z = T0, *G = T0 + 2 * (int64_t)np * nn, *H = T0 + 3 * (int64_t)np * nn,
              *V = T0 + 4 * (int64_t)np * nn;
      MS_TRY(launch_aug_build(ctx, n, np, 3 * n, nullptr, 0, X.a11, s2, X.a12, s2, AUG));        // [I | t_a | rp_a]
      MS_TRY(mm(ctx, n, X.a12, n, s2, X.r + nn, n, s2, AUG, 3 * n, 3 * nn, np, -1.0, 1.0));     // F
      MS_TRY(getrf_aug(ctx, AUG, n, 3 * n, 3 * nn, np, PIV, ctx->d_status, 0));
      MS_TRY(trsm_upper_aug(ctx, AUG, n, 3 * n, 3 * nn, np, Z, 2 * n, s2, ctx->d_status, 0));  // [F^-1 t_a | F^-1 rp_a]
      MS_TRY(mm(ctx, n, X.tp, n, s2, X.r + nn, n, s2, G, n, nn, np, 1.0, 0.0));                 // G = tp_a r_b
      MS_TRY(mm(ctx, n, X.a11 + nn, n, s2, Z, 2 * n, s2, Y.a11, n, nn, np, 1.0, 0.0));          // t
      MS_TRY(launch_axpby(ctx, nn, np, 1.0, X.r, s2, 0.0, nullptr, 0, Y.r, nn));
      MS_TRY(mm(ctx, n, G, n, nn, Z, 2 * n, s2, Y.r, n, nn, np, 1.0, 1.0));                     // r
      MS_TRY(mm(ctx, n, X.a11 + nn, n, s2, Z + n, 2 * n, s2, H, n, nn, np, 1.0, 0.0));
      MS_TRY(launch_axpby(ctx, nn, np, 1.0, X.a12 + nn, s2, 0.0, nullptr, 0, Y.a12, nn));
      MS_TRY(mm(ctx, n, H, n, nn, X.tp + nn, n, s2, Y.a12, n, nn, np, 1.0, 1.0));              // rp
      MS_TRY(launch_axpby(ctx, nn, np, 1.0, X.tp, s2, 0.0, nullptr, 0, V, nn));
      MS_TRY(mm(ctx, n, G, n, nn, Z + n, 2 * n, s2, V, n, nn, np, 1.0, 1.0));
      MS_TRY(mm(ctx, n, V, n, nn, X.tp + nn, n, s2, Y.tp, n, nn, np, 1.0, 0.0));                // tp
    }
    if (nb & 1) {   // the odd last block moves up unchanged
      const int64_t o = (int64_t)(nb - 1) * nn, d = (int64_t)np * nn;
      MS_TRY(launch_axpby(ctx, nn, 1, 1.0, X.a11 + o, 0, 0.0, nullptr, 0, Y.a11 + d, 0));
      MS_TRY(launch_axpby(ctx, nn, 1, 1.0, X.a12 + o, 0, 0.0, nullptr, 0, Y.a12 + d, 0));
      MS_TRY(launch_axpby(ctx, nn, 1, 1.0, X.r + o, 0, 0.0, nullptr, 0, Y.r + d, 0));
      MS_TRY(launch_axpby(ctx, nn, 1, 1.0, X.tp + o, 0, 0.0, nullptr, 0, Y.tp + d, 0));
    }
    nb = np + (nb & 1);
    std::swap(cur, nxt);
    if (mixed) {
      ++levels;
      MS_TRY(cond_pass(*cur, nb, false, &cmax));
      if (cmax > max_cond) {
        mixed = false;
        MS_TRY(cond_pass(*cur, nb, true, nullptr));
      }
    }
  }
  if (mixed) MS_TRY(cond_pass(*cur, 1, true, nullptr));
  const size_t bytes = nn * sizeof(double2);
  MS_HIP(ctx, hipMemcpyAsync(whole->t, cur->a11, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(whole->rp, cur->a12, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(whole->r, cur->r, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(whole->tp, cur->tp, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  *mixed_levels = levels;
  return MS_OK;
}

// ------------------------------------------------------------------------------------------
ms_status ms_kpar_average(ms_ctx ctx, int64_t n_k, int64_t n_e, const double* T, const int64_t* n_open, double* tbar,
                          double* per_channel) {
  if (!ctx) return MS_ERR_ARG;
  if (n_k <= 0 || n_e <= 0) return fail(ctx, MS_ERR_ARG, "n_k and n_e must be positive");
  if (bad_ptr(T) || bad_ptr(n_open) || bad_ptr(tbar) || bad_ptr(per_channel))
    return fail(ctx, MS_ERR_ARG, "NULL pointer argument");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  return launch_kpar_average(ctx, n_k, n_e, T, n_open, tbar, per_channel);
}

}  // extern "C"
