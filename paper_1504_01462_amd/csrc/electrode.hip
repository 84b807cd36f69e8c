// Periodic electrodes (App. B and C): the Bloch states of each electrode cell from its pencil
// (Eq. cmp) by QZ, read at the slice-1 plane where each is largest; their flux and direction;
// the scattering region's S-matrix between the two electrodes' slice-1 planes; the matching of
// Eq. trans in the S-matrix form; T and R from the states' flux matrices.
#include <algorithm>
#include <cmath>
#include <vector>

#include "elem.h"
#include "ms_internal.h"

namespace ms {
namespace {

// workspace slots of this file, above every slot the fold, the cell pencil (ms_bloch_pencil)
// and the star products take, since those run between a request here and its use
enum {
  WE_SEG = 200, WE_WHOLE, WE_EPS2, WE_OVL2, WE_IDX, WE_M, WE_Y, WE_PIV, WE_TMP, WE_EN,
  // the band stage: the batch's pencils (P, Q), their QZ copies and transforms, (alpha, beta),
  // X, one G, the states' (a | b), fluxes and QZ status words
  WB_P = 220, WB_Q, WB_QA, WB_QB, WB_QV, WB_QY, WB_AL, WB_BE, WB_X, WB_G, WB_AB, WB_FL, WB_ST
};
// device bytes the band stage may take for the pencils of one QZ launch
constexpr size_t BANDS_BUDGET = size_t(48) << 30;

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 kz(double e, double eps) {
  const double d = e - eps;
  return d >= 0.0 ? make_double2(sqrt(d), 0.0) : make_double2(0.0, sqrt(-d));
}

// a (n x 2n) and b (n x 2n) of every state c of the pencil: at plane 1 for |lam_c| <= 1
// (a = X_top, b = S21 X_top + S22 X_bot = (Q X)_bot), at plane M+1 otherwise
// (a = S11 X_top + S12 X_bot = (P X)_top, b = X_bot); G = [(P X)_top ; (Q X)_bot] (2n x 2n)
__global__ void k_modes_select(int n, const double2* X, const double2* G, const double2* alpha, const double2* beta,
                               double2* a, double2* b) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = 2 * n;
  if (idx >= (int64_t)n * m) return;
  const int i = (int)(idx / m), c = (int)(idx % m);
  const double al = hypot(alpha[c].x, alpha[c].y), be = beta[c].x;
  const bool grow = al > be;   // |lam| > 1
  a[idx] = grow ? G[(int64_t)i * m + c] : X[(int64_t)i * m + c];
  b[idx] = grow ? X[(int64_t)(n + i) * m + c] : G[(int64_t)(n + i) * m + c];
}

// flux of every state: Re[(a+b)^H K (a-b) + (a-b)^H K^* (a+b)] with K = diag k(E, eps_1)
__global__ __launch_bounds__(256) void k_mode_flux(int n, double energy, const double* eps1, const double2* a,
                                                   const double2* b, double* flux) {
  __shared__ double red[256];
  const int c = blockIdx.x, t = threadIdx.x, m = 2 * n;
  double s = 0.0;
  for (int i = t; i < n; i += 256) {
    const double2 k = kz(energy, eps1[i]);
    const double2 av = a[(int64_t)i * m + c], bv = b[(int64_t)i * m + c];
    const double2 su = make_double2(av.x + bv.x, av.y + bv.y), du = make_double2(av.x - bv.x, av.y - bv.y);
    s += zmul(zconj(su), zmul(k, du)).x + zmul(zconj(du), zmul(zconj(k), su)).x;
  }
  red[t] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) flux[c] = red[0];
}

// dst[:, j] = src[:, idx[j]] for j < cnt (n rows, ld of src ms, of dst ld)
__global__ void k_gather_states(int n, int cnt, const int32_t* idx, const double2* src, int ms, double2* dst, int ld,
                                int coff) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * cnt) return;
  const int i = (int)(e / cnt), j = (int)(e % cnt);
  dst[(int64_t)i * ld + coff + j] = src[(int64_t)i * ms + idx[j]];
}

// T, R from the matching solution y = [tau; rho] (2n x n_in, ld yl) and the states:
//   T = Re Tr[(tau_p^H J_out tau_p) J_in^-1],  R = Re Tr[(rho_p^H J_ref rho_p) J_in^-1]
// with J(u, v) = (A_u + B_u)^H K (A_v - B_v) + (A_u - B_u)^H K^* (A_v + B_v), J_ref = -J of the
// reflected propagating states.  sel: [tp (cnt_t) | rp (cnt_r)] positions of the propagating
// states among the right-going states of the right electrode and the left-going ones of the
// left electrode; states: a, b (n x 2n) of the right electrode's right-going, the left
// electrode's left-going and its incident states, in that column order (ld 3n).
constexpr int EMAX = 24;
__global__ __launch_bounds__(256) void k_electrode_T(int n, int n_in, int cnt_t, int cnt_r, const int32_t* sel,
                                                     double energy, const double* eps_l, const double* eps_r,
                                                     const double2* a, const double2* b, int ld, const double2* y,
                                                     int yl, double* T, double* R) {
  __shared__ double2 jin[EMAX][EMAX + 1], inv[EMAX][EMAX + 1], jm[EMAX][EMAX + 1];
  __shared__ double2 red[256];
  const int t = threadIdx.x;
  // cross flux of columns (cu, cv) of (a, b), channels of slice 1 of the side's cell
  auto cross = [&](const double* eps, int cu, int cv) -> double2 {
    double2 s = make_double2(0.0, 0.0);
    for (int i = t; i < n; i += 256) {
      const double2 k = kz(energy, eps[i]);
      const double2 au = a[(int64_t)i * ld + cu], bu = b[(int64_t)i * ld + cu];
      const double2 av = a[(int64_t)i * ld + cv], bv = b[(int64_t)i * ld + cv];
      const double2 su = make_double2(au.x + bu.x, au.y + bu.y), du = make_double2(au.x - bu.x, au.y - bu.y);
      const double2 sv = make_double2(av.x + bv.x, av.y + bv.y), dv = make_double2(av.x - bv.x, av.y - bv.y);
      const double2 p1 = zmul(zconj(su), zmul(k, dv)), p2 = zmul(zconj(du), zmul(zconj(k), sv));
      s.x += p1.x + p2.x;
      s.y += p1.y + p2.y;
    }
    red[t] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) red[t] = make_double2(red[t].x + red[t + o].x, red[t].y + red[t + o].y);
      __syncthreads();
    }
    const double2 r = red[0];
    __syncthreads();
    return r;
  };
  // J_in (incident states, columns 2n .. 2n + n_in) and its inverse by Gauss-Jordan
  for (int u = 0; u < n_in; ++u)
    for (int v = 0; v < n_in; ++v) {
      const double2 j = cross(eps_l, 2 * n + u, 2 * n + v);
      if (t == 0) jin[u][v] = j;
    }
  __syncthreads();
  if (t == 0) {
    for (int u = 0; u < n_in; ++u)
      for (int v = 0; v < n_in; ++v) inv[u][v] = make_double2(u == v ? 1.0 : 0.0, 0.0);
    for (int c = 0; c < n_in; ++c) {
      int piv = c;
      for (int r = c + 1; r < n_in; ++r)
        if (hypot(jin[r][c].x, jin[r][c].y) > hypot(jin[piv][c].x, jin[piv][c].y)) piv = r;
      for (int v = 0; v < n_in; ++v) {
        const double2 x = jin[c][v], z = inv[c][v];
        jin[c][v] = jin[piv][v];
        inv[c][v] = inv[piv][v];
        jin[piv][v] = x;
        inv[piv][v] = z;
      }
      const double2 d = jin[c][c];
      const double dd = d.x * d.x + d.y * d.y;
      const double2 di = make_double2(d.x / dd, -d.y / dd);
      for (int v = 0; v < n_in; ++v) {
        jin[c][v] = zmul(jin[c][v], di);
        inv[c][v] = zmul(inv[c][v], di);
      }
      for (int r = 0; r < n_in; ++r) {
        if (r == c) continue;
        const double2 f = jin[r][c];
        for (int v = 0; v < n_in; ++v) {
          const double2 p = zmul(f, jin[c][v]), q = zmul(f, inv[c][v]);
          jin[r][v] = make_double2(jin[r][v].x - p.x, jin[r][v].y - p.y);
          inv[r][v] = make_double2(inv[r][v].x - q.x, inv[r][v].y - q.y);
        }
      }
    }
  }
  __syncthreads();
  for (int side = 0; side < 2; ++side) {
    const int cnt = side == 0 ? cnt_t : cnt_r;
    const int32_t* pos = sel + (side == 0 ? 0 : cnt_t);
    const int col0 = side == 0 ? 0 : n;        // state columns: right-going of the right electrode, left-going of the left
    const int row0 = side == 0 ? 0 : n;        // rows of y: tau, rho
    const double* eps = side == 0 ? eps_r : eps_l;
    const double sgn = side == 0 ? 1.0 : -1.0;
    for (int u = 0; u < cnt; ++u)
      for (int v = 0; v < cnt; ++v) {
        const double2 j = cross(eps, col0 + pos[u], col0 + pos[v]);
        if (t == 0) jm[u][v] = make_double2(sgn * j.x, sgn * j.y);
      }
    __syncthreads();
    // Re Tr(w J_in^-1) with w = y_p^H J y_p (n_in x n_in)
    if (t == 0) {
      double tr = 0.0;
      for (int u = 0; u < n_in; ++u)
        for (int v = 0; v < n_in; ++v) {
          double2 s = make_double2(0.0, 0.0);
          for (int p = 0; p < cnt; ++p)
            for (int q = 0; q < cnt; ++q) {
              const double2 yp = y[(int64_t)(row0 + pos[p]) * yl + u], yq = y[(int64_t)(row0 + pos[q]) * yl + v];
              const double2 z = zmul(zconj(yp), zmul(jm[p][q], yq));
              s.x += z.x;
              s.y += z.y;
            }
          tr += zmul(s, inv[v][u]).x;
        }
      if (side == 0) T[0] = tr;
      else R[0] = tr;
    }
    __syncthreads();
  }
}

ms_status check_cell(ms_ctx ctx, const ms_slices* s, const char* name) {
  if (!s) return fail(ctx, MS_ERR_ARG, "%s is NULL", name);
  if (s->n_g <= 0 || s->n_slices <= 0) return fail(ctx, MS_ERR_ARG, "%s: n_g and n_slices must be positive", name);
  if (s->n_g > 2048) return fail(ctx, MS_ERR_UNSUPPORTED, "%s: n_g = %lld > 2048", name, (long long)s->n_g);
  if (!s->dz || !s->eps || !s->ovl || !s->evec)
    return fail(ctx, MS_ERR_ARG, "%s: dz, eps, ovl and evec (the eigenvectors) are required", name);
  return MS_OK;
}

struct Bands {
  const double2 *al, *be, *X, *a, *b;
  std::vector<double2> alh, beh;
  std::vector<double> flux;
};

// The 2n Bloch states of `count` (cell, energy) pairs: each pencil (Eq. cmp) is built with the
// fold's kernels, the pencils' QZ runs as one batch (one workgroup per pencil), then each
// pencil's states are read at their planes (a, b) and their fluxes formed.  Pencils are taken
// in chunks whose eight 2n x 2n buffers fit BANDS_BUDGET; out[k].a, .b stay valid until the next
// call, out[k].al, .be, .X only for the last chunk (count 1: always).
ms_status bands_batch(ms_ctx ctx, int count, const ms_slices* const* cells, const double* energies,
                      std::vector<Bands>& out) {
  const int n = (int)cells[0]->n_g, m = 2 * n;
  const int64_t mm = (int64_t)m * m;
  const size_t big = (size_t)mm * sizeof(double2);
  const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(count, (int64_t)(BANDS_BUDGET / (8 * big))));
  void *P, *Q, *QA, *QB, *QV, *QY, *al, *be, *X, *G, *ab, *fl, *st;
  MS_TRY(workspace(ctx, WB_AB, (size_t)count * 2 * n * m * sizeof(double2), &ab));
  MS_TRY(workspace(ctx, WB_FL, (size_t)count * m * sizeof(double), &fl));
  MS_TRY(workspace(ctx, WB_ST, (size_t)count * sizeof(int32_t), &st));
  std::vector<int32_t> sth(count, 0);
  out.assign(count, Bands{});
  for (int c0 = 0; c0 < count; c0 += chunk) {
    const int cn = std::min(chunk, count - c0);
    // the pencils first: ms_bloch_pencil takes slots of its own, none of WB_*
    MS_TRY(workspace(ctx, WB_P, cn * big, &P));
    MS_TRY(workspace(ctx, WB_Q, cn * big, &Q));
    for (int k = 0; k < cn; ++k)
      MS_TRY(ms_bloch_pencil(ctx, cells[c0 + k], energies[c0 + k], (double2*)P + k * mm, (double2*)Q + k * mm));
    MS_TRY(workspace(ctx, WB_QA, cn * big, &QA));
    MS_TRY(workspace(ctx, WB_QB, cn * big, &QB));
    MS_TRY(workspace(ctx, WB_QV, cn * big, &QV));
    MS_TRY(workspace(ctx, WB_QY, cn * big, &QY));
    MS_TRY(workspace(ctx, WB_AL, (size_t)cn * m * sizeof(double2), &al));
    MS_TRY(workspace(ctx, WB_BE, (size_t)cn * m * sizeof(double2), &be));
    MS_TRY(workspace(ctx, WB_X, cn * big, &X));
    MS_TRY(workspace(ctx, WB_G, big, &G));
    MS_HIP(ctx, hipMemcpyAsync(QA, P, cn * big, hipMemcpyDeviceToDevice, ctx->stream));
    MS_HIP(ctx, hipMemcpyAsync(QB, Q, cn * big, hipMemcpyDeviceToDevice, ctx->stream));
    int32_t* stc = (int32_t*)st + c0;
    MS_TRY(launch_fill_i32(ctx, cn, stc, 0));
    MS_TRY(qz_eig(ctx, m, cn, (double2*)QA, (double2*)QB, (double2*)QV, (double2*)QY, (double2*)al, (double2*)be,
                  (double2*)X, stc));
    for (int k = 0; k < cn; ++k) {
      const int c = c0 + k;
      const double2* Xk = (const double2*)X + k * mm;
      const double2* alk = (const double2*)al + (int64_t)k * m;
      const double2* bek = (const double2*)be + (int64_t)k * m;
      // G = [(P X)_top ; (Q X)_bot]
      GemmArgs g;
      g.M = n; g.N = m; g.K = m;
      g.A = (double2*)P + k * mm; g.lda = m; g.B = Xk; g.ldb = m; g.C = (double2*)G; g.ldc = m;
      MS_TRY(zgemm(ctx, g));
      g.A = (double2*)Q + k * mm + (int64_t)n * m; g.C = (double2*)G + (int64_t)n * m;
      MS_TRY(zgemm(ctx, g));
      double2* a = (double2*)ab + (int64_t)c * 2 * n * m;
      double2* b = a + (int64_t)n * m;
      double* flc = (double*)fl + (int64_t)c * m;
      hipLaunchKernelGGL(k_modes_select, dim3((unsigned)((n * (int64_t)m + 255) / 256)), dim3(256), 0, ctx->stream, n,
                         Xk, (const double2*)G, alk, bek, a, b);
      MS_TRY(check_launch(ctx, "modes select"));
      hipLaunchKernelGGL(k_mode_flux, dim3(m), dim3(256), 0, ctx->stream, n, energies[c], cells[c]->eps + n,
                         (const double2*)a, (const double2*)b, flc);
      MS_TRY(check_launch(ctx, "mode flux"));
      Bands& o = out[c];
      o.al = alk;
      o.be = bek;
      o.X = Xk;
      o.a = a;
      o.b = b;
      o.alh.resize(m);
      o.beh.resize(m);
      MS_HIP(ctx, hipMemcpyAsync(o.alh.data(), alk, m * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
      MS_HIP(ctx, hipMemcpyAsync(o.beh.data(), bek, m * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
    }
  }
  std::vector<double> flh((size_t)count * m);
  MS_HIP(ctx, hipMemcpyAsync(flh.data(), fl, flh.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(sth.data(), st, count * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  MS_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int c = 0; c < count; ++c) {
    if (sth[c] != 0)
      return fail(ctx, (ms_status)sth[c], "QZ of the Bloch pencil at energy %g did not converge", energies[c]);
    out[c].flux.assign(flh.begin() + (int64_t)c * m, flh.begin() + (int64_t)(c + 1) * m);
  }
  return MS_OK;
}

constexpr double PROPAGATING_TOL = 1e-8;   // ||lam| - 1| below this: a propagating Bloch state

struct Dirs {
  std::vector<int32_t> right, left;
  std::vector<char> prop;
};
ms_status directions(ms_ctx ctx, const Bands& bd, int n, const char* name, Dirs* d) {
  const int m = 2 * n;
  d->prop.assign(m, 0);
  for (int c = 0; c < m; ++c) {
    const double al = std::hypot(bd.alh[c].x, bd.alh[c].y), be = bd.beh[c].x;
    const bool prop = std::fabs(al - be) < PROPAGATING_TOL * std::max(al, be);
    d->prop[c] = prop;
    if (prop ? bd.flux[c] > 0.0 : al < be) d->right.push_back(c);
    else d->left.push_back(c);
  }
  if ((int)d->right.size() != n || (int)d->left.size() != n)
    return fail(ctx, MS_ERR_THRESHOLD, "%s: %zu right- and %zu left-going Bloch states, expected %d each (an energy "
                "at a band edge?)", name, d->right.size(), d->left.size(), n);
  return MS_OK;
}

// S(p, p+1) of a two-slice set (slice u with eigenvalues eps_u, thickness dz_u; slice v, dz_v)
// whose overlap is O = Uu^dagger Uv: the interface of two different slice sets
ms_status cross_interface(ms_ctx ctx, int n, const double* eps_u, const double* dz_u, const double2* Uu,
                          const double* eps_v, const double* dz_v, const double2* Uv, double energy, ms_smat* out) {
  const int64_t nn = (int64_t)n * n;
  void *eps2, *ovl2;
  MS_TRY(workspace(ctx, WE_EPS2, (size_t)(4 * n + 2) * sizeof(double), &eps2));
  MS_TRY(workspace(ctx, WE_OVL2, (size_t)3 * nn * sizeof(double2), &ovl2));
  double* e2 = (double*)eps2;
  const size_t row = n * sizeof(double);
  MS_HIP(ctx, hipMemcpyAsync(e2, eps_u, row, hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(e2 + n, eps_u, row, hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(e2 + 2 * n, eps_v, row, hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(e2 + 3 * n, eps_v, row, hipMemcpyDeviceToDevice, ctx->stream));
  double* dz2 = e2 + 4 * n;
  MS_HIP(ctx, hipMemcpyAsync(dz2, dz_u, sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(dz2 + 1, dz_v, sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  GemmArgs g;
  g.M = n; g.N = n; g.K = n;
  g.A = Uu; g.lda = n; g.opA = OP_C;
  g.B = Uv; g.ldb = n;
  g.C = (double2*)ovl2 + nn; g.ldc = n;
  MS_TRY(zgemm(ctx, g));
  const ms_slices pair{n, 2, dz2, e2, ovl2, nullptr};
  return ms_slice_smatrix(ctx, &pair, energy, 1, 2, out);
}

// Eq. trans at one energy from both electrodes' Bloch states (bl, br): the region's S between
// the electrodes' slice-1 planes, the states sorted by direction, the matching solve, and T, R
// written to the device scalars T, R (left as they are without incident states)
ms_status match_one(ms_ctx ctx, const ms_slices* left, const ms_slices* region, const ms_slices* right, double energy,
                    const Bands& bl, const Bands& br, double* T, double* R, int64_t* nin_out) {
  const int n = (int)region->n_g, m = 2 * n, ns = (int)region->n_slices;
  const int64_t nn = (int64_t)n * n;
  Dirs dl, dr;
  MS_TRY(directions(ctx, bl, n, "left electrode", &dl));
  MS_TRY(directions(ctx, br, n, "right electrode", &dr));
  std::vector<int32_t> inc, tp, rp;
  for (int c : dl.right)
    if (dl.prop[c]) inc.push_back(c);
  for (int j = 0; j < n; ++j) {
    if (dr.prop[dr.right[j]]) tp.push_back(j);
    if (dl.prop[dl.left[j]]) rp.push_back(j);
  }
  const int nin = (int)inc.size(), nt = (int)tp.size(), nr = (int)rp.size();
  if (nin > EMAX || nt > EMAX || nr > EMAX)
    return fail(ctx, MS_ERR_UNSUPPORTED, "more than %d propagating states (%d, %d, %d)", EMAX, nin, nt, nr);
  // 2. the region's S between the slice-1 planes of the two electrodes: interfaces
  //    L1 | region 1, region p | p+1, region N | R1 (thickness of R1), star products
  void *seg, *whole;
  MS_TRY(workspace(ctx, WE_SEG, (size_t)(ns + 1) * 4 * nn * sizeof(double2), &seg));
  MS_TRY(workspace(ctx, WE_WHOLE, (size_t)4 * nn * sizeof(double2), &whole));
  std::vector<ms_smat> s(ns + 1);
  for (int i = 0; i <= ns; ++i) {
    double2* p = (double2*)seg + (int64_t)i * 4 * nn;
    s[i] = ms_smat{n, p, p + nn, p + 2 * nn, p + 3 * nn};
  }
  const double2* UL = (const double2*)left->evec;
  const double2* UR = (const double2*)right->evec;
  const double2* UG = (const double2*)region->evec;
  MS_TRY(cross_interface(ctx, n, left->eps + n, left->dz, UL, region->eps + n, region->dz, UG, energy, &s[0]));
  if (ns > 1) MS_TRY(ms_slice_smatrix(ctx, region, energy, 1, ns, s.data() + 1));
  MS_TRY(cross_interface(ctx, n, region->eps + (int64_t)ns * n, region->dz + (ns - 1), UG + (int64_t)(ns - 1) * nn,
                         right->eps + n, right->dz, UR, energy, &s[ns]));
  double2* w = (double2*)whole;
  ms_smat S{n, w, w + nn, w + 2 * nn, w + 3 * nn};
  MS_TRY(ms_star_cascade(ctx, s.data(), ns + 1, MS_PREC_FP64, &S));
  const double2 *S11 = w, *S12 = w + nn, *S21 = w + 2 * nn, *S22 = w + 3 * nn;
  // 3. the states in one block: [right electrode right-going | left electrode left-going |
  //    incident] as a (n x (2n + n_in)) and b, ld 3n
  const int ld = 3 * n;
  void *tmp, *idx;
  MS_TRY(workspace(ctx, WE_TMP, (size_t)2 * n * ld * sizeof(double2), &tmp));
  MS_TRY(workspace(ctx, WE_IDX, (size_t)(2 * n + nin + nt + nr + 1) * sizeof(int32_t), &idx));
  std::vector<int32_t> ih(dr.right);
  ih.insert(ih.end(), dl.left.begin(), dl.left.end());
  ih.insert(ih.end(), inc.begin(), inc.end());
  ih.insert(ih.end(), tp.begin(), tp.end());
  ih.insert(ih.end(), rp.begin(), rp.end());
  MS_TRY(upload(ctx, idx, ih.data(), ih.size() * sizeof(int32_t)));
  const int32_t* id = (const int32_t*)idx;
  double2* SA = (double2*)tmp;            // a of the states
  double2* SB = SA + (int64_t)n * ld;     // b of the states
  auto gather = [&](const Bands& bd, int cnt, const int32_t* ix, int coff) -> ms_status {
    const unsigned gr = (unsigned)(((int64_t)n * cnt + 255) / 256);
    if (cnt == 0) return MS_OK;
    hipLaunchKernelGGL(k_gather_states, dim3(gr), dim3(256), 0, ctx->stream, n, cnt, ix, (const double2*)bd.a, m, SA,
                       ld, coff);
    hipLaunchKernelGGL(k_gather_states, dim3(gr), dim3(256), 0, ctx->stream, n, cnt, ix, (const double2*)bd.b, m, SB,
                       ld, coff);
    return check_launch(ctx, "gather states");
  };
  MS_TRY(gather(br, n, id, 0));
  MS_TRY(gather(bl, n, id + n, n));
  MS_TRY(gather(bl, nin, id + 2 * n, 2 * n));
  // 4. matching: [[Ta - S12 Tb, -S11 Ra], [-S22 Tb, Rb - S21 Ra]] [tau; rho] = [S11 Ia; S21 Ia - Ib]
  const int lm = m + nin;
  void *M, *Y, *piv;
  MS_TRY(workspace(ctx, WE_M, (size_t)m * lm * sizeof(double2), &M));
  MS_TRY(workspace(ctx, WE_Y, (size_t)m * std::max(1, nin) * sizeof(double2), &Y));
  MS_TRY(workspace(ctx, WE_PIV, (size_t)m * sizeof(int32_t) + 16, &piv));
  double2* Mm = (double2*)M;
  auto copy_block = [&](double2* dst, const double2* src, int cols) -> ms_status {   // n rows, ld 3n -> lm
    MS_HIP(ctx, hipMemcpy2DAsync(dst, (size_t)lm * sizeof(double2), src, (size_t)ld * sizeof(double2),
                                 (size_t)cols * sizeof(double2), n, hipMemcpyDeviceToDevice, ctx->stream));
    return MS_OK;
  };
  // top-left Ta, bottom-right Rb, right-hand side top 0 / bottom -Ib (then the GEMMs add the S terms)
  MS_TRY(copy_block(Mm, SA, n));                                     // Ta
  MS_TRY(copy_block(Mm + (int64_t)n * lm + n, SB + n, n));           // Rb
  MS_HIP(ctx, hipMemset2DAsync(Mm + n, (size_t)lm * sizeof(double2), 0, (size_t)(n + nin) * sizeof(double2), n,
                               ctx->stream));                        // top-right and top rhs
  MS_HIP(ctx, hipMemset2DAsync(Mm + (int64_t)n * lm, (size_t)lm * sizeof(double2), 0, (size_t)n * sizeof(double2),
                               n, ctx->stream));                     // bottom-left
  if (nin > 0) {
    MS_TRY(copy_block(Mm + (int64_t)n * lm + m, SB + m, nin));      // Ib, negated below
  }
  auto mm = [&](const double2* A, const double2* B, int cols, double2* C, double2 alpha, double2 beta) {
    GemmArgs g;
    g.M = n; g.N = cols; g.K = n;
    g.A = A; g.lda = n; g.B = B; g.ldb = ld; g.C = C; g.ldc = lm;
    g.alpha = alpha; g.beta = beta;
    return zgemm(ctx, g);
  };
  const double2 ONE = {1.0, 0.0}, MONE = {-1.0, 0.0};
  MS_TRY(mm(S12, SB, n, Mm, MONE, ONE));                              // Ta - S12 Tb
  MS_TRY(mm(S11, SA + n, n, Mm + n, MONE, ONE));                      // -S11 Ra
  MS_TRY(mm(S22, SB, n, Mm + (int64_t)n * lm, MONE, ONE));            // -S22 Tb
  MS_TRY(mm(S21, SA + n, n, Mm + (int64_t)n * lm + n, MONE, ONE));    // Rb - S21 Ra
  if (nin > 0) {
    MS_TRY(mm(S11, SA + m, nin, Mm + m, ONE, ONE));                     // S11 Ia
    MS_TRY(mm(S21, SA + m, nin, Mm + (int64_t)n * lm + m, ONE, MONE));  // S21 Ia - Ib
  }
  if (nin > 0) {
    MS_TRY(getrf_aug(ctx, Mm, m, lm, (int64_t)m * lm, 1, (int32_t*)piv, ctx->d_status, 0));
    MS_TRY(trsm_upper_aug(ctx, Mm, m, lm, (int64_t)m * lm, 1, (double2*)Y, nin, (int64_t)m * nin, ctx->d_status, 0));
  }
  // 5. T and R (zeroed by the caller: nothing to do without incident states)
  *nin_out = nin;
  if (nin == 0) return MS_OK;
  hipLaunchKernelGGL(k_electrode_T, dim3(1), dim3(256), 0, ctx->stream, n, nin, nt, nr, id + 2 * n + nin, energy,
                     left->eps + n, right->eps + n, (const double2*)SA, (const double2*)SB, ld, (const double2*)Y, nin,
                     T, R);
  return check_launch(ctx, "electrode T");
}

// checks shared by the entry points; energies on the host
ms_status check_electrodes(ms_ctx ctx, const ms_slices* left, const ms_slices* region, const ms_slices* right,
                           int64_t n_e, const double* energies) {
  MS_TRY(check_cell(ctx, left, "left"));
  MS_TRY(check_cell(ctx, region, "region"));
  MS_TRY(check_cell(ctx, right, "right"));
  if (left->n_g != region->n_g || right->n_g != region->n_g)
    return fail(ctx, MS_ERR_ARG, "the electrodes and the region need the same basis size");
  if (n_e < 1 || n_e > 32768) return fail(ctx, MS_ERR_ARG, "n_e must be in [1, 32768]");
  if (!energies) return fail(ctx, MS_ERR_ARG, "energies is NULL");
  for (int64_t e = 0; e < n_e; ++e)
    if (!std::isfinite(energies[e])) return fail(ctx, MS_ERR_ARG, "energy %lld is not finite", (long long)e);
  return MS_OK;
}

// both electrodes' bands at every energy in one batch, then the matching energy by energy
ms_status electrode_batch(ms_ctx ctx, const ms_slices* left, const ms_slices* region, const ms_slices* right,
                          int64_t n_e, const double* energies, double* T, double* R, int64_t* n_in) {
  MS_HIP(ctx, hipSetDevice(ctx->device));
  MS_HIP(ctx, hipMemsetAsync(T, 0, n_e * sizeof(double), ctx->stream));
  MS_HIP(ctx, hipMemsetAsync(R, 0, n_e * sizeof(double), ctx->stream));
  std::vector<const ms_slices*> cells;
  std::vector<double> ens;
  for (int side = 0; side < 2; ++side)
    for (int64_t e = 0; e < n_e; ++e) {
      cells.push_back(side == 0 ? right : left);
      ens.push_back(energies[e]);
    }
  std::vector<Bands> bands;
  MS_TRY(bands_batch(ctx, (int)cells.size(), cells.data(), ens.data(), bands));
  std::vector<int64_t> nin(n_e, 0);
  for (int64_t e = 0; e < n_e; ++e) {
    const ms_status st = match_one(ctx, left, region, right, energies[e], bands[n_e + e], bands[e], T + e, R + e,
                                   &nin[e]);
    if (st != MS_OK) {
      ctx->last_error = "energy " + std::to_string((long long)e) + ": " + ctx->last_error;
      return st;
    }
  }
  void* en;
  MS_TRY(workspace(ctx, WE_EN, n_e * sizeof(int64_t), &en));
  MS_TRY(upload(ctx, en, nin.data(), n_e * sizeof(int64_t)));
  MS_HIP(ctx, hipMemcpyAsync(n_in, en, n_e * sizeof(int64_t), hipMemcpyDeviceToDevice, ctx->stream));
  return MS_OK;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" {

ms_status ms_complex_bands(ms_ctx ctx, const ms_slices* cell, double energy, void* alpha, void* beta, void* X) {
  if (!ctx) return MS_ERR_ARG;
  MS_TRY(check_cell(ctx, cell, "cell"));
  if (!std::isfinite(energy)) return fail(ctx, MS_ERR_ARG, "energy must be finite");
  if (!alpha || !beta || !X) return fail(ctx, MS_ERR_ARG, "NULL output pointer");
  MS_HIP(ctx, hipSetDevice(ctx->device));
  std::vector<Bands> bd;
  MS_TRY(bands_batch(ctx, 1, &cell, &energy, bd));
  const int m = 2 * (int)cell->n_g;
  MS_HIP(ctx, hipMemcpyAsync(alpha, bd[0].al, m * sizeof(double2), hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(beta, bd[0].be, m * sizeof(double2), hipMemcpyDeviceToDevice, ctx->stream));
  MS_HIP(ctx, hipMemcpyAsync(X, bd[0].X, (size_t)m * m * sizeof(double2), hipMemcpyDeviceToDevice, ctx->stream));
  return MS_OK;
}

ms_status ms_electrode_transmission(ms_ctx ctx, const ms_slices* left, const ms_slices* region,
                                    const ms_slices* right, double energy, double* T, double* R, int64_t* n_in) {
  if (!ctx) return MS_ERR_ARG;
  MS_TRY(check_electrodes(ctx, left, region, right, 1, &energy));
  if (!T || !R || !n_in) return fail(ctx, MS_ERR_ARG, "NULL output pointer");
  return electrode_batch(ctx, left, region, right, 1, &energy, T, R, n_in);
}

ms_status ms_electrode_transmission_batch(ms_ctx ctx, const ms_slices* left, const ms_slices* region,
                                          const ms_slices* right, int64_t n_e, const double* energies, double* T,
                                          double* R, int64_t* n_in) {
  if (!ctx) return MS_ERR_ARG;
  MS_TRY(check_electrodes(ctx, left, region, right, n_e, energies));
  if (!T || !R || !n_in) return fail(ctx, MS_ERR_ARG, "NULL output pointer");
  return electrode_batch(ctx, left, region, right, n_e, energies, T, R, n_in);
}

}  // extern "C"
