// Per-energy elementwise and reduction kernels of the transmission path.
#include "elem.h"

namespace ms {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// k = sqrt(E - eps) on the branch Im k >= 0;  P = exp(i k dz)
__device__ __forceinline__ double2 kz(double e, double eps) {
  const double d = e - eps;
  return d >= 0.0 ? make_double2(sqrt(d), 0.0) : make_double2(0.0, sqrt(-d));
}
__device__ __forceinline__ double2 prop(double2 k, double dz) {
  const double a = exp(-k.y * dz);
  double s, c;
  sincos(k.x * dz, &s, &c);
  return make_double2(a * c, a * s);
}

// kbuf[e][p][i], pbuf[e][p][i] for p = 0..nrows-1 (nrows = n_slices + 2)
__global__ void k_wavevectors(int n, int nrows, const double* eps, const double* energies, const double* dz,
                              double2* kbuf, double2* pbuf, int64_t sk) {
  const int64_t e = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nrows * n) return;
  const int p = (int)(idx / n);
  const double2 k = kz(energies[e], eps[idx]);
  const double d = (p >= 1 && p <= nrows - 2) ? dz[p - 1] : 0.0;
  kbuf[e * sk + idx] = k;
  pbuf[e * sk + idx] = prop(k, d);
}

__global__ void k_fill_i32(int64_t count, int32_t* v, int32_t value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) v[i] = value;
}

// results of instance i (fold order) to the caller's position perm[i]
__global__ void k_scatter_results(int64_t count, const int64_t* perm, const double* t, const double* r,
                                  const int64_t* no, const int32_t* st, double* T, double* R, int64_t* n_open,
                                  int32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t j = perm[i];
  T[j] = t[i];
  R[j] = r[i];
  n_open[j] = no[i];
  status[j] = st[i];
}

__device__ __forceinline__ void put(double2* d, double2 v) { *d = v; }
__device__ __forceinline__ void put(float2* d, double2 v) { *d = make_float2((float)v.x, (float)v.y); }

// Near-threshold columns of the FP32-MFMA form: per instance e, the first (in index order) at
// most `cap` indices m with |kq_m| < thr, as sel[e][0] = count, sel[e][1..count] = indices
// (one wave per instance, ballots over 64 indices at a time, so the order is fixed).
__global__ __launch_bounds__(64) void k_thresh_select(int n, const double2* kq, int64_t sk, double thr, int cap,
                                                      int32_t* sel) {
  const int64_t e = blockIdx.x;
  const int lane = threadIdx.x;
  const double2* k = kq + e * sk;
  int32_t* out = sel + e * (int64_t)(cap + 1);
  int count = 0;
  for (int m0 = 0; m0 < n && count < cap; m0 += 64) {
    const int m = m0 + lane;
    const bool hit = m < n && (k[m].x * k[m].x + k[m].y * k[m].y) < thr * thr;
    const unsigned long long mask = __ballot(hit);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (hit && count + before < cap) out[1 + count + before] = m;
    count += __popcll(mask);
  }
  if (lane == 0) out[0] = min(count, cap);
}

// A_e = rho^T,  rho^T_ij = P_i k_i Y_ij P_j / k_j  (k, P of slice p+1; Y = Y1 of the state);
// with sel (FP32 form) the selected near-threshold columns are left out (zero)
template <typename OutT>
__global__ void k_prologue(int n, const double2* Y, int64_t ldy, int64_t sY, const double2* kq, const double2* pq,
                           int64_t sk, const int32_t* sel, int cap, OutT* Aop) {
  const int64_t e = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  const double2* k = kq + e * sk;
  const double2* P = pq + e * sk;
  bool skip = false;
  if (sel) {
    const int32_t* se = sel + e * (int64_t)(cap + 1);
    for (int c = 0; c < se[0]; ++c) skip = skip || se[1 + c] == j;
  }
  const double2 y = Y[e * sY + (int64_t)i * ldy + j];
  put(Aop + e * (int64_t)n * n + idx,
      skip ? make_double2(0.0, 0.0) : cdiv(cmul(cmul(cmul(P[i], k[i]), y), P[j]), k[j]));
}

// With C+- = O^T K_p +- K_{p+1} O^T (elementwise: O_ji (kp_j +- kq_i)) and W = rho^T [C- | C+ off
// its diagonal] from the interface product:
//   M_e[:, 0:n]  = Phi_A^T = C+ + rho^T C-
//   M_e[:, n:2n] = Phi_B^T = C- + rho^T C+   (the diagonal part rho^T_ij C+_jj added here, in FP64)
// rho^T is formed again from Y in FP64, and so are the terms of the near-threshold columns m in
// sel (left out of the FP32 product): rho^T_im C-_mj and rho^T_im C+_mj (m != j).  O^T read
// through a 32 x 32 LDS tile; W may be null (first interface: rho = 0).
__global__ __launch_bounds__(256) void k_epilogue(int n, const double2* O, const double2* Wg, const double2* kp,
                                                  const double2* kq, const double2* pq, int64_t sk, const double2* Y,
                                                  int64_t ldy, int64_t sY, const int32_t* sel, int cap, double2* M,
                                                  int64_t ldm, int64_t sM) {
  __shared__ double2 tile[32][33];
  const int64_t e = blockIdx.z;
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // O^T(i, j) = O(j, i): load O rows bj.., cols bi..
  for (int r = ty; r < 32; r += 8) {
    const int oi = bj + r, oj = bi + tx;
    tile[r][tx] = (oi < n && oj < n) ? O[(int64_t)oi * n + oj] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const double2* k_p = kp + e * sk;
  const double2* k_q = kq + e * sk;
  const double2* P = pq + e * sk;
  const int32_t* se = sel ? sel + e * (int64_t)(cap + 1) : nullptr;
  const int nsel = se ? se[0] : 0;
  for (int r = ty; r < 32; r += 8) {
    const int i = bi + r, j = bj + tx;
    if (i >= n || j >= n) continue;
    const double2 ot = tile[tx][r];
    const double2 cp = cmul(ot, cadd(k_p[j], k_q[i]));
    const double2 cm = cmul(ot, csub(k_p[j], k_q[i]));
    double2* Mr = M + e * sM + (int64_t)i * ldm;
    if (!Wg) {
      Mr[j] = cp;
      Mr[n + j] = cm;
      continue;
    }
    const double2* W = Wg + e * 2 * (int64_t)n * n + (int64_t)i * 2 * n;
    const double2* Yi = Y + e * sY + (int64_t)i * ldy;
    const double2 pk = cmul(P[i], k_q[i]);
    const double2 rho = cdiv(cmul(cmul(pk, Yi[j]), P[j]), k_q[j]);
    const double2 cpd = cmul(O[(int64_t)j * n + j], cadd(k_p[j], k_q[j]));
    double2 wm = W[j], wp = cadd(W[n + j], cmul(rho, cpd));
    for (int c = 0; c < nsel; ++c) {
      const int m = se[1 + c];
      const double2 rm = cdiv(cmul(cmul(pk, Yi[m]), P[m]), k_q[m]);
      const double2 ojm = O[(int64_t)j * n + m];
      wm = cadd(wm, cmul(rm, cmul(ojm, csub(k_p[j], k_q[m]))));
      if (m != j) wp = cadd(wp, cmul(rm, cmul(ojm, cadd(k_p[j], k_q[m]))));
    }
    Mr[j] = cadd(cp, wm);
    Mr[n + j] = cadd(cm, wp);
  }
}

// M_e[:, 2n + c] = P_i T~_ic,  T~ = unit columns e_{ch_c} (first interface) or 2 K Y2
__global__ void k_tcols(int n, int n_o, const int32_t* ch, const double2* Y, int64_t ldy, int64_t sY, int y_off,
                        const double2* kq, const double2* pq, int64_t sk, int first, double2* M, int64_t ldm,
                        int64_t sM) {
  const int64_t e = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n_o) return;
  const int i = (int)(idx / n_o), c = (int)(idx % n_o);
  double2 v;
  if (first) {
    v = make_double2(ch[c] == i ? 1.0 : 0.0, 0.0);
  } else {
    const double2 k = kq[e * sk + i];
    v = cmul(make_double2(2.0 * k.x, 2.0 * k.y), Y[e * sY + (int64_t)i * ldy + y_off + c]);
  }
  M[e * sM + (int64_t)i * ldm + 2 * n + c] = cmul(pq[e * sk + i], v);
}

// Sums (and a minimum, a count) over the 256 threads of a workgroup: butterfly shuffles inside
// each wave, then the four wave results in a fixed order, so the result is the same every run.
struct TRPart {
  double t, r, m;
  int o;
};
__device__ __forceinline__ TRPart block_reduce_tr(TRPart v, TRPart* wave_part) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.t += __shfl_xor(v.t, off, 64);
    v.r += __shfl_xor(v.r, off, 64);
    v.m = fmin(v.m, __shfl_xor(v.m, off, 64));
    v.o += __shfl_xor(v.o, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wave_part[wave] = v;
  __syncthreads();
  TRPart s = wave_part[0];
  for (int w = 1; w < 4; ++w) {
    s.t += wave_part[w].t;
    s.r += wave_part[w].r;
    s.m = fmin(s.m, wave_part[w].m);
    s.o += wave_part[w].o;
  }
  return s;
}

// T, R, N_open of the fused path from the final state (Y1 = K^-1 r^T K, Y2 = (2K)^-1 t^T)
__global__ __launch_bounds__(256) void k_batch_T(int n, int n_o, const int32_t* ch, const double* energies,
                                                 const double* eps_l, const double* eps_r, const double2* Y,
                                                 int64_t ldy, int64_t sY, double* T, double* R, int64_t* n_open,
                                                 int32_t* status) {
  __shared__ TRPart wp[4];
  const int64_t e = blockIdx.x;
  const int t = threadIdx.x;
  const double E = energies[e];
  const double2* Yb = Y + e * sY;
  double tt = 0.0, rr = 0.0, mind = 1e300;
  int no = 0;
  for (int i = t; i < n; i += 256) {
    mind = fmin(mind, fmin(fabs(E - eps_l[i]), fabs(E - eps_r[i])));
    if (eps_l[i] < E) no++;
  }
  for (int64_t idx = t; idx < (int64_t)n * n_o; idx += 256) {
    const int j = (int)(idx / n_o), c = (int)(idx % n_o);
    if (eps_l[j] < E && eps_r[ch[c]] < E) {
      const double kl = sqrt(E - eps_l[j]), kr = sqrt(E - eps_r[ch[c]]);
      tt += 4.0 * kr * kl * cabs2(Yb[(int64_t)j * ldy + n + c]);
    }
  }
  for (int64_t idx = t; idx < (int64_t)n * n; idx += 256) {
    const int a = (int)(idx / n), b = (int)(idx % n);
    if (eps_l[a] < E && eps_l[b] < E) {
      const double ka = sqrt(E - eps_l[a]), kb = sqrt(E - eps_l[b]);
      rr += (ka / kb) * cabs2(Yb[(int64_t)a * ldy + b]);
    }
  }
  const TRPart sum = block_reduce_tr(TRPart{tt, rr, mind, no}, wp);
  if (t == 0) {
    T[e] = sum.t;
    R[e] = sum.r;
    n_open[e] = sum.o;
    int32_t code = 0;
    if (sum.m < 1e-10) code = MS_ERR_THRESHOLD;
    else if (!isfinite(sum.t) || !isfinite(sum.r)) code = MS_ERR_NONFINITE;
    if (code) atomicCAS(status + e, 0, code);
  }
}

// T, R, N_open from a whole-junction S-matrix (t = S11, r = S21)
__global__ __launch_bounds__(256) void k_whole_T(int n, double E, const double2* t, const double2* r,
                                                 const double* eps_l, const double* eps_r, double* T, double* R,
                                                 int64_t* n_open, int32_t* status) {
  __shared__ TRPart wp[4];
  const int tid = threadIdx.x;
  double tt = 0.0, rr = 0.0, mind = 1e300;
  int no = 0;
  for (int i = tid; i < n; i += 256) {
    mind = fmin(mind, fmin(fabs(E - eps_l[i]), fabs(E - eps_r[i])));
    if (eps_l[i] < E) no++;
  }
  for (int64_t idx = tid; idx < (int64_t)n * n; idx += 256) {
    const int i = (int)(idx / n), j = (int)(idx % n);
    if (eps_l[j] < E) {
      const double kj = sqrt(E - eps_l[j]);
      if (eps_r[i] < E) tt += (sqrt(E - eps_r[i]) / kj) * cabs2(t[idx]);
      if (eps_l[i] < E) rr += (sqrt(E - eps_l[i]) / kj) * cabs2(r[idx]);
    }
  }
  const TRPart sum = block_reduce_tr(TRPart{tt, rr, mind, no}, wp);
  if (tid == 0) {
    T[0] = sum.t;
    R[0] = sum.r;
    n_open[0] = sum.o;
    if (sum.m < 1e-10) atomicCAS(status, 0, (int32_t)MS_ERR_THRESHOLD);
    else if (!isfinite(sum.t) || !isfinite(sum.r)) atomicCAS(status, 0, (int32_t)MS_ERR_NONFINITE);
  }
}

// aug_b = [X | I | Y], Xc_b = X, Yc_b = Y for interface p = p0 + b
//   X_ij = O_ij (kp_i + kq_j) / (2 kp_i),  Y_ij = O_ij (kp_i - kq_j) / (2 kp_i)
__global__ void k_xy(int n, const double2* ovl, const double2* kbuf, int p0, double2* aug, double2* Xc, double2* Yc) {
  const int64_t b = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  const int64_t nn = (int64_t)n * n;
  const double2 o = ovl[(p0 + b) * nn + idx];
  const double2 kp = kbuf[(p0 + b) * n + i], kq = kbuf[(p0 + b + 1) * n + j];
  const double2 h = cdiv(o, make_double2(2.0 * kp.x, 2.0 * kp.y));
  const double2 x = cmul(h, cadd(kp, kq)), y = cmul(h, csub(kp, kq));
  double2* A = aug + b * 3 * nn + (int64_t)i * 3 * n;
  A[j] = x;
  A[n + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  A[2 * n + j] = y;
  Xc[b * nn + idx] = x;
  Yc[b * nn + idx] = y;
}

// S11 = P X^-1, S12 = -P X^-1 Y P, S22 = (X - Y X^-1 Y) P   (Z = [X^-1 | X^-1 Y], Xc = X - Y X^-1 Y)
__global__ void k_smat_finish(int n, const double2* Z, const double2* Xc, const double2* pbuf, int p0, double2* tout,
                              double2* rpout, double2* tpout) {
  const int64_t b = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  const int64_t nn = (int64_t)n * n;
  const double2* P = pbuf + (p0 + b + 1) * n;
  const double2* Zr = Z + b * 2 * nn + (int64_t)i * 2 * n;
  tout[b * nn + idx] = cmul(P[i], Zr[j]);
  const double2 s12 = cmul(cmul(P[i], Zr[n + j]), P[j]);
  rpout[b * nn + idx] = make_double2(-s12.x, -s12.y);
  tpout[b * nn + idx] = cmul(Xc[b * nn + idx], P[j]);
}

// aug = [I | t_a | rp_a]  (the GEMM then adds -rp_a r_b to the first block)
__global__ void k_star_aug(int n, const double2* ta, const double2* rpa, double2* aug) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  double2* A = aug + (int64_t)i * 3 * n;
  A[j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  A[n + j] = ta[idx];
  A[2 * n + j] = rpa[idx];
}

__global__ void k_to_c64(int64_t count, const double2* in, float2* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) out[idx] = make_float2((float)in[idx].x, (float)in[idx].y);
}

__global__ void k_nonfinite_scan(int64_t count, const double2* v, int32_t* status) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count && !(isfinite(v[idx].x) && isfinite(v[idx].y))) atomicCAS(status, 0, (int32_t)MS_ERR_NONFINITE);
}

// k_par average of T and transmission per open channel (one thread per energy)
__global__ void k_kpar_average(int64_t n_k, int64_t n_e, const double* T, const int64_t* n_open, double* tbar,
                               double* per_channel) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_e) return;
  double st = 0.0;
  int64_t so = 0;
  for (int64_t k = 0; k < n_k; ++k) {
    st += T[k * n_e + e];
    so += n_open[k * n_e + e];
  }
  tbar[e] = st / (double)n_k;
  per_channel[e] = so > 0 ? st / (double)so : 0.0;
}

// Transfer blocks of App. A, Eq. (transfer): I11 = X P^-1, I12 = Y P for interfaces
// p0 + b, with X, Y as in k_xy and P = diag e^{i k^{p+1} dz_{p+1}}.
__global__ void k_transfer_blocks(int n, const double2* ovl, const double2* kbuf, const double2* pbuf, int p0,
                                  double2* I11, double2* I12) {
  const int64_t b = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  const int64_t nn = (int64_t)n * n;
  const double2 o = ovl[(p0 + b) * nn + idx];
  const double2 kp = kbuf[(p0 + b) * n + i], kq = kbuf[(p0 + b + 1) * n + j];
  const double2 h = cdiv(o, make_double2(2.0 * kp.x, 2.0 * kp.y));
  const double2 x = cmul(h, cadd(kp, kq)), y = cmul(h, csub(kp, kq));
  const double2 P = pbuf[(p0 + b + 1) * n + j];
  I11[b * nn + idx] = cdiv(x, P);
  I12[b * nn + idx] = cmul(y, P);
}

// aug[b] (n x w, w = 2n or 3n) = [first | I | ...]: first = src[b] (stride s_src) or, when
// src is null, the identity; the block after it is the identity when ident2 is set,
// else copied from src2[b]; a third block (w = 3n) is copied from src3[b].
__global__ void k_aug_build(int n, int w, const double2* src, int64_t s_src, const double2* src2, int64_t s_src2,
                            const double2* src3, int64_t s_src3, double2* aug) {
  const int64_t b = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  double2* A = aug + b * (int64_t)n * w + (int64_t)i * w;
  const double2 id = make_double2(i == j ? 1.0 : 0.0, 0.0);
  A[j] = src ? src[b * s_src + idx] : id;
  A[n + j] = src2 ? src2[b * s_src2 + idx] : id;
  if (w == 3 * n) A[2 * n + j] = src3[b * s_src3 + idx];
}

// out[b] = alpha a[b] + beta c[b] (element strides per batch entry)
__global__ void k_axpby(int64_t nn, double alpha, const double2* a, int64_t s_a, double beta, const double2* c,
                        int64_t s_c, double2* out, int64_t s_o) {
  const int64_t b = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  const double2 x = a[b * s_a + idx];
  double2 v = make_double2(alpha * x.x, alpha * x.y);
  if (c) {
    const double2 y = c[b * s_c + idx];
    v.x += beta * y.x;
    v.y += beta * y.y;
  }
  out[b * s_o + idx] = v;
}

// 1-norm (largest column sum of |a_ij|) of each n x n matrix (row stride ld, batch stride s)
__global__ __launch_bounds__(256) void k_norm1(int n, const double2* A, int64_t ld, int64_t s, double* out) {
  __shared__ double red[256];
  const int64_t b = blockIdx.x;
  const double2* M = A + b * s;
  double best = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    double sum = 0.0;
    for (int i = 0; i < n; ++i) sum += hypot(M[(int64_t)i * ld + j].x, M[(int64_t)i * ld + j].y);
    best = fmax(best, sum);
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = red[0];
}

inline unsigned blocks(int64_t count) { return (unsigned)((count + 255) / 256); }

// ---- first variation of T (gradient with respect to the slice potentials) -------------

// The open-channel system of the out-states, from the reduced whole S: r (n x n), tpc = t'[:, orr]
// (n x nr), trow = t[orr, :] (nr x n), rpo = r'[orr, orr] (nr x nr).  Rows/cols [0, nl) are the
// left lead's open channels ol, [nl, nl + nr) the right lead's.  aug = [[r_OO, t'_OR], [t_RO,
// r'_RR] | 0; I] (row-major, width nl + 2 nr).  blockIdx.y = energy b: channel tables olt, ort
// hold [b][nl] and [b][nr] entries, -1 for padding (an identity row and column, zero right-hand
// side); the states of energy b are b * s_st elements after energy 0's.
__global__ void k_grad_open_system(int n, int nl, int nr, const int32_t* olt, const int32_t* ort, const double2* r,
                                   const double2* tpc, const double2* trow, const double2* rpo, int64_t s_st,
                                   double2* aug) {
  const int m = nl + nr, w = m + nr;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * w) return;
  const int64_t b = blockIdx.y;
  const int32_t* ol = olt + b * nl;
  const int32_t* orr = ort + b * nr;
  r += b * s_st;
  tpc += b * s_st;
  trow += b * s_st;
  rpo += b * s_st;
  const int i = idx / w, j = idx % w;
  const bool row_open = i < nl ? ol[i] >= 0 : orr[i - nl] >= 0;
  double2 v = make_double2(0.0, 0.0);
  if (j < m) {
    const bool col_open = j < nl ? ol[j] >= 0 : orr[j - nl] >= 0;
    if (!row_open || !col_open) v = make_double2(i == j ? 1.0 : 0.0, 0.0);   // padding
    else if (i < nl && j < nl) v = r[(int64_t)ol[i] * n + ol[j]];
    else if (i < nl) v = tpc[(int64_t)ol[i] * nr + (j - nl)];
    else if (j < nl) v = trow[(int64_t)(i - nl) * n + ol[j]];
    else v = rpo[(int64_t)(i - nl) * nr + (j - nl)];
  } else if (row_open && i >= nl && (i - nl) == (j - m)) {
    v = make_double2(1.0, 0.0);
  }
  aug[b * m * w + idx] = v;
}

// dst[i][j] = src[rows ? rows[i] : i][cols ? cols[j] : j] for i < nrow, j < ncol (an index
// of -1 gives 0); blockIdx.y = batch entry b, every pointer advanced by its stride times b
__global__ void k_gather2(int nrow, int ncol, const int32_t* rows, int64_t s_rows, const int32_t* cols,
                          int64_t s_cols, const double2* src, int64_t lds, int64_t s_src, double2* dst, int64_t ldd,
                          int64_t s_dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nrow * ncol) return;
  const int64_t b = blockIdx.y;
  const int i = (int)(e / ncol), j = (int)(e % ncol);
  const int si = rows ? rows[b * s_rows + i] : i, sj = cols ? cols[b * s_cols + j] : j;
  dst[b * s_dst + (int64_t)i * ldd + j] =
      (si < 0 || sj < 0) ? make_double2(0.0, 0.0) : src[b * s_src + (int64_t)si * lds + sj];
}

// dst[rows[i]][:] = src[i][:] (n columns) for i < nrow; the other rows of dst are left as they are
__global__ void k_scatter_rows(int nrow, int n, const int32_t* rows, const double2* src, double2* dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nrow * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  if (rows[i] < 0) return;   // a padded row
  dst[(int64_t)rows[i] * n + j] = src[e];
}

// dst[:, c] = src[:, idx[c]] for c < nc (n rows; row-major, leading dims lds, ldd); idx < 0: zero
__global__ void k_gather_cols(int n, int nc, const int32_t* idx, const double2* src, int64_t lds, double2* dst,
                              int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * nc) return;
  const int i = (int)(e / nc), c = (int)(e % nc);
  const int s = idx[c];
  dst[(int64_t)i * ldd + c] = s >= 0 ? src[(int64_t)i * lds + s] : make_double2(0.0, 0.0);
}

// int_{-w}^{0} e^{i kappa s} ds
__device__ __forceinline__ double2 exp_integral(double2 kap, double w) {
  const double2 x = make_double2(-kap.y * w, kap.x * w);       // i kappa w
  if (x.x * x.x + x.y * x.y < 1e-16) return make_double2(w * (1.0 - 0.5 * x.x), -0.5 * w * x.y);
  const double em = exp(-x.x);                                 // e^{-x}
  const double2 one_minus = make_double2(1.0 - em * cos(-x.y), -em * sin(-x.y));
  const double2 ik = make_double2(-kap.y, kap.x);
  return cdiv(one_minus, ik);
}

// conj(M) of one slice, n x n row-major:
//   M_nm = sum_j P1_nj (a_mj E(k_m - k*_n) + b_mj E(-k_m - k*_n)) + P2_nj (a_mj E(k_m + k*_n) + b_mj E(-k_m + k*_n))
// with P1 = conj(C) w, P2 = conj(D) w (n x nl), a, b the in-states' amplitudes (n x nl),
// k the slice's wavevectors, w its thickness.
__global__ void k_grad_m(int n, int nl, const double2* kall, int64_t s_k, double width, const double2* p1all,
                         const double2* p2all, int64_t s_p, const double2* aall, int64_t lda, int64_t s_a,
                         const double2* ball, int64_t ldb, int64_t s_b, double2* mcall, int64_t s_m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int64_t bb = blockIdx.y;
  const double2* k = kall + bb * s_k;
  const double2* p1 = p1all + bb * s_p;
  const double2* p2 = p2all + bb * s_p;
  const double2* a = aall + bb * s_a;
  const double2* b = ball + bb * s_b;
  double2* mc = mcall + bb * s_m;
  const int row = (int)(e / n), col = (int)(e % n);
  const double2 kn = cconj(k[row]), km = k[col];
  const double2 e1 = exp_integral(make_double2(km.x - kn.x, km.y - kn.y), width);
  const double2 e2 = exp_integral(make_double2(-km.x - kn.x, -km.y - kn.y), width);
  const double2 e3 = exp_integral(make_double2(km.x + kn.x, km.y + kn.y), width);
  const double2 e4 = exp_integral(make_double2(-km.x + kn.x, -km.y + kn.y), width);
  double2 acc = make_double2(0.0, 0.0);
  for (int j = 0; j < nl; ++j) {
    const double2 aj = a[(int64_t)col * lda + j], bj = b[(int64_t)col * ldb + j];
    const double2 u = cadd(cmul(aj, e1), cmul(bj, e2));
    const double2 v = cadd(cmul(aj, e3), cmul(bj, e4));
    acc = cadd(acc, cadd(cmul(p1[(int64_t)row * nl + j], u), cmul(p2[(int64_t)row * nl + j], v)));
  }
  mc[e] = cconj(acc);
}

// P = conj(C) w: P_nj = sum_i conj(C_ni) w_ij, w_ij = conj(t_ij) / (2 i k_j)  (i over the right
// lead's open channels, j over the left lead's: ol[j] < 0 or a padded row i (trow = 0 there)
// contribute nothing; trow = the open rows t[orr, :] of the whole S).  blockIdx.y = energy b.
__global__ void k_grad_p(int n, int nl, int nr, const double2* c, int64_t ldc, int64_t s_c, const double2* d,
                         int64_t ldd, int64_t s_d, const double2* trow, int64_t s_trow, const int32_t* ol, int64_t s_ol,
                         const double2* kl, int64_t s_kl, double2* p1, double2* p2, int64_t s_p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * nl) return;
  const int64_t b = blockIdx.y;
  const int row = (int)(e / nl), j = (int)(e % nl);
  const int oj = ol[b * s_ol + j];
  double2 s1 = make_double2(0.0, 0.0), s2 = make_double2(0.0, 0.0);
  if (oj >= 0) {
    const double2 kj = kl[b * s_kl + oj];
    const double2 den = make_double2(-2.0 * kj.y, 2.0 * kj.x);   // 2 i k_j
    for (int i = 0; i < nr; ++i) {
      const double2 w = cdiv(cconj(trow[b * s_trow + (int64_t)i * n + oj]), den);
      s1 = cadd(s1, cmul(cconj(c[b * s_c + (int64_t)row * ldc + i]), w));
      s2 = cadd(s2, cmul(cconj(d[b * s_d + (int64_t)row * ldd + i]), w));
    }
  }
  p1[b * s_p + e] = s1;
  p2[b * s_p + e] = s2;
}

// the first n columns of an n-row matrix (leading dim ld) set to the identity
// P = [[S11, S12], [0, I]], Q = [[I, 0], [S21, S22]] (2n x 2n row-major) from the blocks of a
// cell S-matrix, (S11, S12, S21, S22) = (t, rp, r, tp)
__global__ void k_bloch_pencil(int n, const double2* t, const double2* rp, const double2* r, const double2* tp,
                               double2* P, double2* Q) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = 2 * (int64_t)n;
  if (e >= m * m) return;
  const int i = (int)(e / m), j = (int)(e % m);
  const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);
  if (i < n) {
    P[e] = j < n ? t[(int64_t)i * n + j] : rp[(int64_t)i * n + (j - n)];
    Q[e] = j < n ? (i == j ? one : zero) : zero;
  } else {
    P[e] = j < n ? zero : (i == j ? one : zero);
    Q[e] = j < n ? r[(int64_t)(i - n) * n + j] : tp[(int64_t)(i - n) * n + (j - n)];
  }
}

__global__ void k_eye(int n, int64_t ld, double2* dst, int64_t s_dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  dst[blockIdx.y * s_dst + (int64_t)i * ld + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
}

// g[q(a,b)] += conj(Kc_ab)
__global__ void k_grad_scatter(int64_t nn, const int32_t* q, const double2* kcall, int64_t s_kc, double* gall,
                               int64_t s_g) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const int64_t qi = q[e];
  const double2 v = kcall[blockIdx.y * s_kc + e];
  double* g = gall + blockIdx.y * s_g;
  atomicAdd(g + 2 * qi, v.x);
  atomicAdd(g + 2 * qi + 1, -v.y);
}

}  // namespace

ms_status launch_wavevectors(ms_ctx ctx, int n, int nrows, int n_e, const double* eps, const double* energies_dev,
                             const double* dz, double2* kbuf, double2* pbuf, int64_t sk) {
  if (sk <= 0) sk = (int64_t)nrows * n;
  hipLaunchKernelGGL(k_wavevectors, dim3(blocks((int64_t)nrows * n), n_e), dim3(256), 0, ctx->stream, n, nrows, eps,
                     energies_dev, dz, kbuf, pbuf, sk);
  return check_launch(ctx, "wavevectors");
}

ms_status launch_fill_i32(ms_ctx ctx, int64_t count, int32_t* v, int32_t value) {
  if (count <= 0) return MS_OK;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, ctx->stream, count, v, value);
  return check_launch(ctx, "fill");
}

ms_status launch_scatter_results(ms_ctx ctx, int64_t count, const int64_t* perm, const double* t, const double* r,
                                 const int64_t* no, const int32_t* st, double* T, double* R, int64_t* n_open,
                                 int32_t* status) {
  if (count <= 0) return MS_OK;
  hipLaunchKernelGGL(k_scatter_results, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, ctx->stream, count, perm,
                     t, r, no, st, T, R, n_open, status);
  return check_launch(ctx, "scatter results");
}

ms_status launch_thresh_select(ms_ctx ctx, int n, int n_e, const double2* kq, int64_t sk, double thr, int cap,
                               int32_t* sel) {
  hipLaunchKernelGGL(k_thresh_select, dim3(n_e), dim3(64), 0, ctx->stream, n, kq, sk, thr, cap, sel);
  return check_launch(ctx, "threshold select");
}

ms_status launch_prologue(ms_ctx ctx, int n, int n_e, const double2* Y, int64_t ldy, int64_t sY, const double2* kq,
                          const double2* pq, int64_t sk, const int32_t* sel, int cap, void* Aop, bool fp32) {
  if (fp32)
    hipLaunchKernelGGL((k_prologue<float2>), dim3(blocks((int64_t)n * n), n_e), dim3(256), 0, ctx->stream, n, Y, ldy,
                       sY, kq, pq, sk, sel, cap, static_cast<float2*>(Aop));
  else
    hipLaunchKernelGGL((k_prologue<double2>), dim3(blocks((int64_t)n * n), n_e), dim3(256), 0, ctx->stream, n, Y,
                       ldy, sY, kq, pq, sk, sel, cap, static_cast<double2*>(Aop));
  return check_launch(ctx, "prologue");
}

ms_status launch_epilogue(ms_ctx ctx, int n, int n_e, const double2* O, const double2* Wg, const double2* kp,
                          const double2* kq, const double2* pq, int64_t sk, const double2* Y, int64_t ldy, int64_t sY,
                          const int32_t* sel, int cap, double2* M, int64_t ldm, int64_t sM) {
  dim3 g((n + 31) / 32, (n + 31) / 32, n_e);
  hipLaunchKernelGGL(k_epilogue, g, dim3(256), 0, ctx->stream, n, O, Wg, kp, kq, pq, sk, Y, ldy, sY, sel, cap, M, ldm,
                     sM);
  return check_launch(ctx, "epilogue");
}

ms_status launch_tcols(ms_ctx ctx, int n, int n_o, int n_e, const int32_t* ch, const double2* Y, int64_t ldy,
                       int64_t sY, int y_off, const double2* kq, const double2* pq, int64_t sk, int first, double2* M,
                       int64_t ldm, int64_t sM) {
  if (n_o <= 0) return MS_OK;
  hipLaunchKernelGGL(k_tcols, dim3(blocks((int64_t)n * n_o), n_e), dim3(256), 0, ctx->stream, n, n_o, ch, Y, ldy, sY,
                     y_off, kq, pq, sk, first, M, ldm, sM);
  return check_launch(ctx, "tcols");
}

ms_status launch_batch_T(ms_ctx ctx, int n, int n_o, int n_e, const int32_t* ch, const double* energies,
                         const double* eps_l, const double* eps_r, const double2* Y, int64_t ldy, int64_t sY, double* T,
                         double* R, int64_t* n_open, int32_t* status) {
  hipLaunchKernelGGL(k_batch_T, dim3(n_e), dim3(256), 0, ctx->stream, n, n_o, ch, energies, eps_l, eps_r, Y, ldy, sY,
                     T, R, n_open, status);
  return check_launch(ctx, "batch T");
}

ms_status launch_whole_T(ms_ctx ctx, int n, double E, const double2* t, const double2* r, const double* eps_l,
                         const double* eps_r, double* T, double* R, int64_t* n_open, int32_t* status) {
  hipLaunchKernelGGL(k_whole_T, dim3(1), dim3(256), 0, ctx->stream, n, E, t, r, eps_l, eps_r, T, R, n_open, status);
  return check_launch(ctx, "whole T");
}

ms_status launch_xy(ms_ctx ctx, int n, int nb, const double2* ovl, const double2* kbuf, int p0, double2* aug,
                    double2* Xc, double2* Yc) {
  hipLaunchKernelGGL(k_xy, dim3(blocks((int64_t)n * n), nb), dim3(256), 0, ctx->stream, n, ovl, kbuf, p0, aug, Xc, Yc);
  return check_launch(ctx, "xy");
}

ms_status launch_smat_finish(ms_ctx ctx, int n, int nb, const double2* Z, const double2* Xc, const double2* pbuf,
                             int p0, double2* tout, double2* rpout, double2* tpout) {
  hipLaunchKernelGGL(k_smat_finish, dim3(blocks((int64_t)n * n), nb), dim3(256), 0, ctx->stream, n, Z, Xc, pbuf, p0,
                     tout, rpout, tpout);
  return check_launch(ctx, "smat finish");
}

ms_status launch_star_aug(ms_ctx ctx, int n, const double2* ta, const double2* rpa, double2* aug) {
  hipLaunchKernelGGL(k_star_aug, dim3(blocks((int64_t)n * n)), dim3(256), 0, ctx->stream, n, ta, rpa, aug);
  return check_launch(ctx, "star aug");
}

ms_status launch_to_c64(ms_ctx ctx, int64_t count, const double2* in, float2* out) {
  hipLaunchKernelGGL(k_to_c64, dim3(blocks(count)), dim3(256), 0, ctx->stream, count, in, out);
  return check_launch(ctx, "to c64");
}

ms_status launch_kpar_average(ms_ctx ctx, int64_t n_k, int64_t n_e, const double* T, const int64_t* n_open,
                               double* tbar, double* per_channel) {
  hipLaunchKernelGGL(k_kpar_average, dim3(blocks(n_e)), dim3(256), 0, ctx->stream, n_k, n_e, T, n_open, tbar,
                     per_channel);
  return check_launch(ctx, "kpar average");
}

ms_status launch_nonfinite_scan(ms_ctx ctx, int64_t count, const double2* v, int32_t* status) {
  hipLaunchKernelGGL(k_nonfinite_scan, dim3(blocks(count)), dim3(256), 0, ctx->stream, count, v, status);
  return check_launch(ctx, "nonfinite scan");
}


ms_status launch_transfer_blocks(ms_ctx ctx, int n, int nb, const double2* ovl, const double2* kbuf,
                                 const double2* pbuf, int p0, double2* I11, double2* I12) {
  hipLaunchKernelGGL(k_transfer_blocks, dim3(blocks((int64_t)n * n), nb), dim3(256), 0, ctx->stream, n, ovl, kbuf,
                     pbuf, p0, I11, I12);
  return check_launch(ctx, "transfer blocks");
}

ms_status launch_aug_build(ms_ctx ctx, int n, int nb, int w, const double2* src, int64_t s_src, const double2* src2,
                           int64_t s_src2, const double2* src3, int64_t s_src3, double2* aug) {
  hipLaunchKernelGGL(k_aug_build, dim3(blocks((int64_t)n * n), nb), dim3(256), 0, ctx->stream, n, w, src, s_src, src2,
                     s_src2, src3, s_src3, aug);
  return check_launch(ctx, "augmented matrix");
}

ms_status launch_axpby(ms_ctx ctx, int64_t nn, int nb, double alpha, const double2* a, int64_t s_a, double beta,
                       const double2* c, int64_t s_c, double2* out, int64_t s_o) {
  hipLaunchKernelGGL(k_axpby, dim3(blocks(nn), nb), dim3(256), 0, ctx->stream, nn, alpha, a, s_a, beta, c, s_c, out,
                     s_o);
  return check_launch(ctx, "axpby");
}

ms_status launch_norm1(ms_ctx ctx, int n, int nb, const double2* A, int64_t ld, int64_t s, double* out) {
  hipLaunchKernelGGL(k_norm1, dim3(nb), dim3(256), 0, ctx->stream, n, A, ld, s, out);
  return check_launch(ctx, "1-norm");
}


ms_status launch_grad_open_system(ms_ctx ctx, int n, int nl, int nr, const int32_t* olt, const int32_t* ort,
                                  const double2* r, const double2* tpc, const double2* trow, const double2* rpo,
                                  int64_t s_st, double2* aug, int batch) {
  const int total = (nl + nr) * (nl + 2 * nr);
  hipLaunchKernelGGL(k_grad_open_system, dim3((total + 255) / 256, batch), dim3(256), 0, ctx->stream, n, nl, nr, olt,
                     ort, r, tpc, trow, rpo, s_st, aug);
  return check_launch(ctx, "gradient open system");
}

ms_status launch_gather2(ms_ctx ctx, int nrow, int ncol, const int32_t* rows, const int32_t* cols,
                         const double2* src, int64_t lds, double2* dst, int64_t ldd, int batch, int64_t s_rows,
                         int64_t s_cols, int64_t s_src, int64_t s_dst) {
  if ((int64_t)nrow * ncol <= 0 || batch <= 0) return MS_OK;
  hipLaunchKernelGGL(k_gather2, dim3(blocks((int64_t)nrow * ncol), batch), dim3(256), 0, ctx->stream, nrow, ncol, rows,
                     s_rows, cols, s_cols, src, lds, s_src, dst, ldd, s_dst);
  return check_launch(ctx, "gather");
}

ms_status launch_scatter_rows(ms_ctx ctx, int nrow, int n, const int32_t* rows, const double2* src, double2* dst) {
  if ((int64_t)nrow * n <= 0) return MS_OK;
  hipLaunchKernelGGL(k_scatter_rows, dim3(blocks((int64_t)nrow * n)), dim3(256), 0, ctx->stream, nrow, n, rows, src,
                     dst);
  return check_launch(ctx, "scatter rows");
}

ms_status launch_gather_cols(ms_ctx ctx, int n, int nc, const int32_t* idx, const double2* src, int64_t lds,
                             double2* dst, int64_t ldd) {
  hipLaunchKernelGGL(k_gather_cols, dim3(blocks((int64_t)n * nc)), dim3(256), 0, ctx->stream, n, nc, idx, src, lds,
                     dst, ldd);
  return check_launch(ctx, "gather columns");
}

ms_status launch_grad_p(ms_ctx ctx, int n, int nl, int nr, const double2* c, int64_t ldc, int64_t s_c,
                        const double2* d, int64_t ldd, int64_t s_d, const double2* trow, int64_t s_trow,
                        const int32_t* ol, int64_t s_ol, const double2* kl, int64_t s_kl, double2* p1, double2* p2,
                        int64_t s_p, int batch) {
  hipLaunchKernelGGL(k_grad_p, dim3(blocks((int64_t)n * nl), batch), dim3(256), 0, ctx->stream, n, nl, nr, c, ldc, s_c,
                     d, ldd, s_d, trow, s_trow, ol, s_ol, kl, s_kl, p1, p2, s_p);
  return check_launch(ctx, "gradient weights");
}

ms_status launch_grad_m(ms_ctx ctx, int n, int nl, const double2* k, int64_t s_k, double width, const double2* p1,
                        const double2* p2, int64_t s_p, const double2* a, int64_t lda, int64_t s_a, const double2* b,
                        int64_t ldb, int64_t s_b, double2* mc, int64_t s_m, int batch) {
  hipLaunchKernelGGL(k_grad_m, dim3(blocks((int64_t)n * n), batch), dim3(256), 0, ctx->stream, n, nl, k, s_k, width, p1,
                     p2, s_p, a, lda, s_a, b, ldb, s_b, mc, s_m);
  return check_launch(ctx, "gradient slice integrals");
}

ms_status launch_bloch_pencil(ms_ctx ctx, int n, const double2* t, const double2* rp, const double2* r,
                              const double2* tp, double2* P, double2* Q) {
  hipLaunchKernelGGL(k_bloch_pencil, dim3(blocks(4 * (int64_t)n * n)), dim3(256), 0, ctx->stream, n, t, rp, r, tp, P,
                     Q);
  return check_launch(ctx, "Bloch pencil");
}

ms_status launch_eye(ms_ctx ctx, int n, int64_t ld, double2* dst, int batch, int64_t s_dst) {
  hipLaunchKernelGGL(k_eye, dim3(blocks((int64_t)n * n), batch), dim3(256), 0, ctx->stream, n, ld, dst, s_dst);
  return check_launch(ctx, "identity");
}

ms_status launch_grad_scatter(ms_ctx ctx, int64_t nn, const int32_t* q, const double2* kc, int64_t s_kc, double* g,
                              int64_t s_g, int batch) {
  hipLaunchKernelGGL(k_grad_scatter, dim3(blocks(nn), batch), dim3(256), 0, ctx->stream, nn, q, kc, s_kc, g, s_g);
  return check_launch(ctx, "gradient scatter");
}

}  // namespace ms
