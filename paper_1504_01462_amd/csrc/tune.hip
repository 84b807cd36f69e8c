// Tile shapes of the fold's GEMMs, chosen by timing.
//
// For a basis size n_g and a batch of systems, ms_autotune builds synthetic augmented
// systems of the fold's shape (n_g x (2 n_g + n_open)) and interface-product operands,
// times the LU factorisation + back substitution with every combination of the two tile
// edges for the LU's trailing update and its in-panel / U12 products, and the interface
// product with both edges (64: 64 x 64 tiles, 128: 128 x 64 tiles), and records the fastest
// per role for that n_g.  The two tile shapes accumulate every element in the same order, so
// the choice changes run time only.
#include <algorithm>
#include <cmath>

#include "ms_internal.h"

namespace ms {
namespace {

// counter-hash value in [-1, 1) (splitmix64 finaliser)
__device__ __forceinline__ double hval(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// batch row-major rows x cols complex matrices (stride s) of hashed entries, plus `diag`
// on the leading diagonal
__global__ void k_synthetic(int rows, int cols, int64_t s, int batch, double diag, uint64_t seed, double2* M) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)rows * cols;
  if (idx >= per * batch) return;
  const int64_t b = idx / per, r = idx % per;
  const int i = (int)(r / cols), j = (int)(r % cols);
  double2 v = make_double2(hval(seed + 2 * (uint64_t)idx), hval(seed + 2 * (uint64_t)idx + 1));
  if (i == j) v.x += diag;
  M[b * s + r] = v;
}

ms_status fill(ms_ctx ctx, int rows, int cols, int64_t s, int batch, double diag, uint64_t seed, void* M) {
  const int64_t total = (int64_t)rows * cols * batch;
  hipLaunchKernelGGL(k_synthetic, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, ctx->stream, rows, cols, s,
                     batch, diag, seed, static_cast<double2*>(M));
  return check_launch(ctx, "synthetic operands");
}

ms_ctx_s::Tiles* entry(ms_ctx ctx, int64_t n) {
  for (auto& t : ctx->tiles)
    if (t.n == n) return &t;
  ctx->tiles.push_back(ms_ctx_s::Tiles{n, 0, 0, 0});
  return &ctx->tiles.back();
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" {

ms_status ms_set_tiles(ms_ctx ctx, int64_t n_g, const ms_tiles* tiles) {
  if (!ctx) return MS_ERR_ARG;
  if (!tiles) return fail(ctx, MS_ERR_ARG, "tiles is NULL");
  if (n_g < 1) return fail(ctx, MS_ERR_ARG, "n_g must be >= 1");
  for (int v : {tiles->iface, tiles->lu_update, tiles->lu_inner})
    if (v != 0 && v != 64 && v != 128) return fail(ctx, MS_ERR_ARG, "tile edge %d is not 0, 64 or 128", v);
  ms_ctx_s::Tiles* t = entry(ctx, n_g);
  t->iface = tiles->iface;
  t->lu_update = tiles->lu_update;
  t->lu_inner = tiles->lu_inner;
  return MS_OK;
}

ms_status ms_autotune(ms_ctx ctx, int64_t n_g, int64_t n_open, int64_t batch, ms_tiles* chosen, double* times_ms) {
  if (!ctx) return MS_ERR_ARG;
  if (n_g < 1 || n_g > 4096) return fail(ctx, MS_ERR_ARG, "n_g must be in [1, 4096]");
  if (n_open < 0 || n_open > n_g) return fail(ctx, MS_ERR_ARG, "n_open must be in [0, n_g]");
  if (batch < 1) return fail(ctx, MS_ERR_ARG, "batch must be >= 1");
  if (!chosen) return fail(ctx, MS_ERR_ARG, "chosen is NULL");
  if (ctx->capturing) return fail(ctx, MS_ERR_UNSUPPORTED, "autotune inside a graph capture");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  const int n = (int)n_g, nb = (int)std::min<int64_t>(batch, 64);
  const int ncols = 2 * n + (int)n_open, nrhs = ncols - n;
  const int64_t sM = (int64_t)n * ncols, sY = (int64_t)n * nrhs, nn = (int64_t)n * n;
  void *M, *Y, *piv, *st, *A, *B, *C;
  MS_TRY(workspace(ctx, 50, (size_t)nb * sM * sizeof(double2), &M));
  MS_TRY(workspace(ctx, 51, (size_t)nb * sY * sizeof(double2), &Y));
  MS_TRY(workspace(ctx, 52, (size_t)nb * n * sizeof(int32_t), &piv));
  MS_TRY(workspace(ctx, 53, (size_t)nb * sizeof(int32_t), &st));
  void* K;
  MS_TRY(workspace(ctx, 54, (size_t)nb * nn * sizeof(double2), &A));
  MS_TRY(workspace(ctx, 55, (size_t)nn * sizeof(double2), &B));
  MS_TRY(workspace(ctx, 56, (size_t)nb * 2 * nn * sizeof(double2), &C));
  MS_TRY(workspace(ctx, 57, (size_t)nb * 2 * n * sizeof(double2), &K));
  MS_TRY(lu_reserve(ctx, n, ncols, nb));
  hipEvent_t e0, e1;
  MS_HIP(ctx, hipEventCreate(&e0));
  MS_HIP(ctx, hipEventCreate(&e1));
  ms_ctx_s::Tiles* t = entry(ctx, n);
  const ms_ctx_s::Tiles saved = *t;
  const int64_t saved_n = ctx->tile_n;
  ctx->tile_n = n;
  const uint32_t saved_mask = ctx->prof_mask;
  ctx->prof_mask = 0;
  ms_status s = MS_OK;
  auto timed = [&](auto body) -> double {   // best of two runs, ms
    double best = 1e300;
    for (int r = 0; r < 2 && s == MS_OK; ++r) {
      s = body(true);   // set-up outside the timed region
      if (s != MS_OK) break;
      hipError_t e = hipEventRecord(e0, ctx->stream);
      if (e == hipSuccess) s = body(false);
      if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms_ = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms_, e0, e1);
      if (e != hipSuccess && s == MS_OK) s = hip_fail(ctx, e, "autotune timing");
      best = std::min(best, (double)ms_);
    }
    return best;
  };
  // the LU factorisation + back substitution of nb synthetic systems per (update, inner) edges
  double lu_ms[2][2] = {{0, 0}, {0, 0}};
  const int edge[2] = {64, 128};
  for (int a = 0; a < 2 && s == MS_OK; ++a)
    for (int c = 0; c < 2 && s == MS_OK; ++c) {
      t->lu_update = edge[a];
      t->lu_inner = edge[c];
      lu_ms[a][c] = timed([&](bool setup) -> ms_status {
        if (setup) return fill(ctx, n, ncols, sM, nb, 4.0 * n, 12345u, M);
        MS_TRY(getrf_aug(ctx, static_cast<double2*>(M), n, ncols, sM, nb, static_cast<int32_t*>(piv),
                         static_cast<int32_t*>(st), 1));
        return trsm_upper_aug(ctx, static_cast<double2*>(M), n, ncols, sM, nb, static_cast<double2*>(Y), nrhs, sY,
                              static_cast<int32_t*>(st), 1);
      });
    }
  // the interface product W = A [C- | C+] of nb systems sharing one O (B generated from O and
  // each system's two wavevector rows)
  double if_ms[2] = {0, 0};
  for (int a = 0; a < 2 && s == MS_OK; ++a) {
    t->iface = edge[a];
    if_ms[a] = timed([&](bool setup) -> ms_status {
      if (setup) {
        MS_TRY(fill(ctx, n * nb, n, 0, 1, 0.0, 777u, A));
        MS_TRY(fill(ctx, 2 * nb, n, 0, 1, 1.0, 555u, K));
        return fill(ctx, n, n, 0, 1, 0.0, 999u, B);
      }
      GemmArgs g;
      g.M = n; g.N = 2 * n; g.K = n;
      g.A = A; g.lda = n; g.sA = nn; g.opA = OP_N;
      g.B = B; g.ldb = n; g.sB = 0; g.opB = OP_T;
      g.C = static_cast<double2*>(C); g.ldc = 2 * n; g.sC = 2 * nn;
      g.batch = nb;
      g.kp = static_cast<const double2*>(K);
      g.kq = static_cast<const double2*>(K) + n;
      g.sk = 2 * n;
      g.prof = PC_IFACE_GEMM;
      return zgemm(ctx, g);
    });
  }
  ctx->prof_mask = saved_mask;
  ctx->tile_n = saved_n;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != MS_OK) {
    *t = saved;
    return s;
  }
  int ba = 0, bc = 0;
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c)
      if (lu_ms[a][c] < lu_ms[ba][bc]) { ba = a; bc = c; }
  t->lu_update = edge[ba];
  t->lu_inner = edge[bc];
  t->iface = if_ms[1] <= if_ms[0] ? 128 : 64;
  chosen->iface = t->iface;
  chosen->lu_update = t->lu_update;
  chosen->lu_inner = t->lu_inner;
  if (times_ms) {   // [lu 64/64, 64/128, 128/64, 128/128, iface 64, iface 128]
    times_ms[0] = lu_ms[0][0]; times_ms[1] = lu_ms[0][1]; times_ms[2] = lu_ms[1][0]; times_ms[3] = lu_ms[1][1];
    times_ms[4] = if_ms[0]; times_ms[5] = if_ms[1];
  }
  return MS_OK;
}

}  // extern "C"
