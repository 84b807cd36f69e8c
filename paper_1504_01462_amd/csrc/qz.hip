// Generalized non-Hermitian eigenproblem A x = lam B x of a batch of complex pencils (the
// electrodes' Bloch pencils of App. B, Eq. cmp) by the QZ iteration: unitary U, V with
// U^H A V = S, U^H B V = T upper triangular, eigenvalues lam_k = S_kk / T_kk kept as the
// pairs (alpha_k, beta_k) = (S_kk, T_kk), so states that change by more than FP64 spans over one
// cell (beta ~ 0 or alpha ~ 0) stay exact pairs.  Right eigenvectors x_k = V y_k with
// (beta_k S - alpha_k T) y_k = 0 by back substitution.
//
// One workgroup per pencil, matrices in global memory (row-major, leading dimension n):
//   1. B = U1 R by Householder reflections, applied to A from the left;
//   2. Hessenberg-triangular reduction: Givens rotations from the left zero A below its
//      subdiagonal column by column, each followed by a rotation from the right that removes
//      the fill it leaves below the diagonal of B (both applied to V from the right);
//   3. implicit single-shift QZ sweeps on the active block, the shift being the eigenvalue of
//      the trailing 2 x 2 pencil nearer its last diagonal ratio; negligible subdiagonal entries
//      of A split the block; negligible diagonal entries of B (infinite eigenvalues) are chased
//      to the bottom of the block and deflated there;
//   4. Y by back substitution, one eigenvector per thread.
// Rotation parameters are formed by one thread and shared through LDS; every rotation is
// applied by all threads of the workgroup along the rows or columns it touches.
#include <cmath>

#include "ms_internal.h"

namespace ms {
namespace {

constexpr int QZ_THREADS = 256;
constexpr double QZ_EPS = 2.220446049250313e-16;

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double zabs(double2 a) { return hypot(a.x, a.y); }
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.y + b.x * r;
  return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__device__ __forceinline__ double2 zsqrt(double2 z) {
  const double m = zabs(z);
  if (m == 0.0) return make_double2(0.0, 0.0);
  const double re = sqrt(0.5 * (m + fabs(z.x)));
  const double im = 0.5 * z.y / re;
  return z.x >= 0.0 ? make_double2(re, im) : make_double2(fabs(im), z.y >= 0.0 ? re : -re);
}

struct Rot {
  double c;
  double2 s;
};

// G = [[c, s], [-conj(s), c]] with G [a; b] = [r; 0]
__device__ __forceinline__ Rot rot_zero_second(double2 a, double2 b) {
  const double aa = zabs(a), bb = zabs(b);
  if (bb == 0.0) return Rot{1.0, make_double2(0.0, 0.0)};
  if (aa == 0.0) return Rot{0.0, make_double2(1.0, 0.0)};
  const double r = hypot(aa, bb);
  const double2 ua = zscale(1.0 / aa, a);
  return Rot{aa / r, zscale(1.0 / r, zmul(ua, zconj(b)))};
}
// Z = [[c, s], [-conj(s), c]] with [x, y] Z = [0, r]
__device__ __forceinline__ Rot rot_zero_first(double2 x, double2 y) {
  const double xx = zabs(x), yy = zabs(y);
  if (xx == 0.0) return Rot{1.0, make_double2(0.0, 0.0)};
  if (yy == 0.0) return Rot{0.0, make_double2(1.0, 0.0)};
  const double r = hypot(xx, yy);
  const double c = yy / r;
  return Rot{c, zscale(c, zconj(zdiv(x, y)))};
}

// rows r1, r2 of M, columns [c0, c1): [M_r1; M_r2] <- G [M_r1; M_r2]
__device__ __forceinline__ void rot_rows(double2* M, int n, int r1, int r2, int c0, int c1, Rot g) {
  double2* p = M + (int64_t)r1 * n;
  double2* q = M + (int64_t)r2 * n;
  for (int k = c0 + (int)threadIdx.x; k < c1; k += QZ_THREADS) {
    const double2 a = p[k], b = q[k];
    p[k] = zadd(zscale(g.c, a), zmul(g.s, b));
    q[k] = zsub(zscale(g.c, b), zmul(zconj(g.s), a));
  }
}
// columns c1, c2 of M, rows [r0, r1): [M_c1, M_c2] <- [M_c1, M_c2] Z
__device__ __forceinline__ void rot_cols(double2* M, int n, int c1, int c2, int r0, int r1, Rot z) {
  for (int k = r0 + (int)threadIdx.x; k < r1; k += QZ_THREADS) {
    double2* row = M + (int64_t)k * n;
    const double2 x = row[c1], y = row[c2];
    row[c1] = zsub(zscale(z.c, x), zmul(zconj(z.s), y));
    row[c2] = zadd(zmul(z.s, x), zscale(z.c, y));
  }
}

__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < QZ_THREADS / 64; ++w) s += red[w];
  return s;
}

// Frobenius norm of the n x n matrix M
__device__ double frob(const double2* M, int n, double* red) {
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < (int64_t)n * n; k += QZ_THREADS) s += M[k].x * M[k].x + M[k].y * M[k].y;
  return sqrt(block_sum(s, red));
}

__global__ __launch_bounds__(QZ_THREADS) void k_qz(int n, double2* Aall, double2* Ball, double2* Vall,
                                                   double2* Yall, double2* alpha, double2* beta, int32_t* status,
                                                   int max_iter_per_eig) {
  extern __shared__ double2 hv[];   // Householder vector [n]
  __shared__ double red[QZ_THREADS / 64];
  __shared__ Rot rot;
  __shared__ double2 wsh;
  __shared__ int flag;
  const int64_t p = blockIdx.x;
  const int64_t nn = (int64_t)n * n;
  double2* A = Aall + p * nn;
  double2* B = Ball + p * nn;
  double2* V = Vall + p * nn;
  double2* Y = Yall + p * nn;
  const int t = threadIdx.x;

  for (int64_t k = t; k < nn; k += QZ_THREADS) V[k] = make_double2((k / n) == (k % n) ? 1.0 : 0.0, 0.0);

  // ---- 1. Householder QR of B, applied to A from the left
  for (int j = 0; j < n - 1; ++j) {
    double s = 0.0;
    for (int i = j + 1 + t; i < n; i += QZ_THREADS) {
      const double2 x = B[(int64_t)i * n + j];
      s += x.x * x.x + x.y * x.y;
    }
    const double tail = block_sum(s, red);
    if (tail == 0.0) continue;   // column already reduced (every thread sees the same sum)
    const double2 x0 = B[(int64_t)j * n + j];
    const double nrm = sqrt(tail + x0.x * x0.x + x0.y * x0.y);
    const double a0 = zabs(x0);
    const double2 ph = a0 > 0.0 ? zscale(1.0 / a0, x0) : make_double2(1.0, 0.0);
    // v = x + ph nrm e_j (no cancellation), H = I - 2 v v^H / (v^H v)
    const double2 v0 = zadd(x0, zscale(nrm, ph));
    const double vv = tail + v0.x * v0.x + v0.y * v0.y;
    for (int i = j + t; i < n; i += QZ_THREADS) hv[i] = (i == j) ? v0 : B[(int64_t)i * n + j];
    __syncthreads();
    const double tau = 2.0 / vv;
    // apply to the columns j..n-1 of B and all columns of A
    for (int m = 0; m < 2; ++m) {
      double2* M = m == 0 ? B : A;
      const int c0 = m == 0 ? j : 0;
      for (int c = c0 + t; c < n; c += QZ_THREADS) {
        double2 w = make_double2(0.0, 0.0);
        for (int i = j; i < n; ++i) w = zadd(w, zmul(zconj(hv[i]), M[(int64_t)i * n + c]));
        w = zscale(tau, w);
        for (int i = j; i < n; ++i) M[(int64_t)i * n + c] = zsub(M[(int64_t)i * n + c], zmul(hv[i], w));
      }
    }
    __syncthreads();
    for (int i = j + 1 + t; i < n; i += QZ_THREADS) B[(int64_t)i * n + j] = make_double2(0.0, 0.0);
    __syncthreads();
  }

  // ---- 2. Hessenberg-triangular reduction
  for (int j = 0; j + 2 < n; ++j) {
    for (int i = n - 1; i >= j + 2; --i) {
      __syncthreads();
      if (t == 0) rot = rot_zero_second(A[(int64_t)(i - 1) * n + j], A[(int64_t)i * n + j]);
      __syncthreads();
      const Rot g = rot;
      rot_rows(A, n, i - 1, i, j, n, g);
      rot_rows(B, n, i - 1, i, i - 1, n, g);
      __syncthreads();
      if (t == 0) {
        A[(int64_t)i * n + j] = make_double2(0.0, 0.0);
        rot = rot_zero_first(B[(int64_t)i * n + i - 1], B[(int64_t)i * n + i]);
      }
      __syncthreads();
      const Rot z = rot;
      rot_cols(B, n, i - 1, i, 0, i + 1, z);
      rot_cols(A, n, i - 1, i, 0, n, z);
      rot_cols(V, n, i - 1, i, 0, n, z);
      __syncthreads();
      if (t == 0) B[(int64_t)i * n + i - 1] = make_double2(0.0, 0.0);
    }
  }
  __syncthreads();

  // ---- 3. QZ iteration
  const double anorm = frob(A, n, red), bnorm = frob(B, n, red);
  const double atol = QZ_EPS * fmax(anorm, 1e-300), btol = QZ_EPS * fmax(bnorm, 1e-300);
  int ihi = n - 1, iter = 0, since = 0;
  const int max_iter = max_iter_per_eig * n;
  while (ihi >= 0) {
    __syncthreads();
    if (ihi == 0) break;
    // infinite eigenvalue at the bottom: deflate through a column rotation
    if (zabs(B[(int64_t)ihi * n + ihi]) <= btol) {
      __syncthreads();
      if (t == 0) {
        B[(int64_t)ihi * n + ihi] = make_double2(0.0, 0.0);
        rot = rot_zero_first(A[(int64_t)ihi * n + ihi - 1], A[(int64_t)ihi * n + ihi]);
      }
      __syncthreads();
      const Rot z = rot;
      rot_cols(A, n, ihi - 1, ihi, 0, ihi + 1, z);
      rot_cols(B, n, ihi - 1, ihi, 0, ihi, z);
      rot_cols(V, n, ihi - 1, ihi, 0, n, z);
      __syncthreads();
      if (t == 0) A[(int64_t)ihi * n + ihi - 1] = make_double2(0.0, 0.0);
      --ihi;
      since = 0;
      continue;
    }
    // negligible subdiagonal at the bottom: a 1 x 1 block deflates
    {
      const double2 sub = A[(int64_t)ihi * n + ihi - 1];
      const double d = zabs(A[(int64_t)ihi * n + ihi]) + zabs(A[(int64_t)(ihi - 1) * n + ihi - 1]);
      if (zabs(sub) <= fmax(atol, QZ_EPS * d)) {
        __syncthreads();
        if (t == 0) A[(int64_t)ihi * n + ihi - 1] = make_double2(0.0, 0.0);
        --ihi;
        since = 0;
        continue;
      }
    }
    // the active block [ilo, ihi]: up from ihi to a negligible subdiagonal
    int ilo = ihi - 1;
    while (ilo > 0) {
      const double2 sub = A[(int64_t)ilo * n + ilo - 1];
      const double d = zabs(A[(int64_t)ilo * n + ilo]) + zabs(A[(int64_t)(ilo - 1) * n + ilo - 1]);
      if (zabs(sub) <= fmax(atol, QZ_EPS * d)) break;
      --ilo;
    }
    __syncthreads();
    if (ilo > 0 && t == 0) A[(int64_t)ilo * n + ilo - 1] = make_double2(0.0, 0.0);
    // a negligible diagonal entry of B inside the block: chase it down to ihi
    int jz = -1;
    for (int j = ilo; j < ihi; ++j)
      if (zabs(B[(int64_t)j * n + j]) <= btol) {
        jz = j;
        break;
      }
    if (jz >= 0) {
      __syncthreads();
      if (t == 0) B[(int64_t)jz * n + jz] = make_double2(0.0, 0.0);
      for (int j = jz; j < ihi; ++j) {
        __syncthreads();
        if (t == 0) rot = rot_zero_second(B[(int64_t)j * n + j + 1], B[(int64_t)(j + 1) * n + j + 1]);
        __syncthreads();
        const Rot g = rot;
        rot_rows(B, n, j, j + 1, j + 1, n, g);
        rot_rows(A, n, j, j + 1, j > ilo ? j - 1 : j, n, g);
        __syncthreads();
        if (t == 0) B[(int64_t)(j + 1) * n + j + 1] = make_double2(0.0, 0.0);
        if (j > ilo) {   // A[j+1][j-1] filled: a column rotation restores the Hessenberg form
          __syncthreads();
          if (t == 0) rot = rot_zero_first(A[(int64_t)(j + 1) * n + j - 1], A[(int64_t)(j + 1) * n + j]);
          __syncthreads();
          const Rot z = rot;
          rot_cols(A, n, j - 1, j, 0, j + 2, z);
          rot_cols(B, n, j - 1, j, 0, j + 1, z);
          rot_cols(V, n, j - 1, j, 0, n, z);
          __syncthreads();
          if (t == 0) A[(int64_t)(j + 1) * n + j - 1] = make_double2(0.0, 0.0);
        }
      }
      continue;   // the zero is at ihi now: deflated at the top of the loop
    }
    if (++iter > max_iter) {
      if (t == 0) atomicCAS(status + p, 0, (int32_t)MS_ERR_NOCONV);
      break;
    }
    ++since;
    // shift: eigenvalue of the trailing 2 x 2 pencil nearer A_hh / B_hh
    double2 sigma;
    {
      const int h = ihi;
      const double2 a11 = A[(int64_t)(h - 1) * n + h - 1], a12 = A[(int64_t)(h - 1) * n + h];
      const double2 a21 = A[(int64_t)h * n + h - 1], a22 = A[(int64_t)h * n + h];
      const double2 b11 = B[(int64_t)(h - 1) * n + h - 1], b12 = B[(int64_t)(h - 1) * n + h];
      const double2 b22 = B[(int64_t)h * n + h];
      // M = B22^-1 A22 (B22 upper triangular, its diagonal above btol here)
      const double2 m21 = zdiv(a21, b22), m22 = zdiv(a22, b22);
      const double2 m11 = zdiv(zsub(a11, zmul(b12, m21)), b11);
      const double2 m12 = zdiv(zsub(a12, zmul(b12, m22)), b11);
      const double2 tr = zadd(m11, m22);
      const double2 half = zscale(0.5, tr);
      const double2 disc = zsqrt(zsub(zmul(half, half), zsub(zmul(m11, m22), zmul(m12, m21))));
      const double2 l1 = zadd(half, disc), l2 = zsub(half, disc);
      sigma = zabs(zsub(l1, m22)) <= zabs(zsub(l2, m22)) ? l1 : l2;
      if (since % 10 == 0) {   // exceptional shift
        const double e = zabs(zdiv(a21, b11));
        sigma = zadd(m22, make_double2(0.7 * e, 0.3 * e));
      }
    }
    // first rotation from (A - sigma B) e_ilo
    __syncthreads();
    if (t == 0) {
      const double2 x = zsub(A[(int64_t)ilo * n + ilo], zmul(sigma, B[(int64_t)ilo * n + ilo]));
      const double2 y = A[(int64_t)(ilo + 1) * n + ilo];
      rot = rot_zero_second(x, y);
    }
    __syncthreads();
    for (int k = ilo; k < ihi; ++k) {
      if (k > ilo) {   // remove the bulge A[k+1][k-1]
        __syncthreads();
        if (t == 0) rot = rot_zero_second(A[(int64_t)k * n + k - 1], A[(int64_t)(k + 1) * n + k - 1]);
        __syncthreads();
      }
      const Rot g = rot;
      rot_rows(A, n, k, k + 1, k > ilo ? k - 1 : k, n, g);
      rot_rows(B, n, k, k + 1, k, n, g);
      __syncthreads();
      if (t == 0) {
        if (k > ilo) A[(int64_t)(k + 1) * n + k - 1] = make_double2(0.0, 0.0);
        rot = rot_zero_first(B[(int64_t)(k + 1) * n + k], B[(int64_t)(k + 1) * n + k + 1]);
      }
      __syncthreads();
      const Rot z = rot;
      rot_cols(A, n, k, k + 1, 0, min(k + 3, ihi + 1), z);
      rot_cols(B, n, k, k + 1, 0, k + 2, z);
      rot_cols(V, n, k, k + 1, 0, n, z);
      __syncthreads();
      if (t == 0) B[(int64_t)(k + 1) * n + k] = make_double2(0.0, 0.0);
    }
  }
  __syncthreads();

  // ---- eigenvalue pairs: beta real and >= 0 (the row of S, T scaled by a unit phase)
  for (int k = t; k < n; k += QZ_THREADS) {
    const double2 sk = A[(int64_t)k * n + k], tk = B[(int64_t)k * n + k];
    const double bt = zabs(tk);
    const double2 ph = bt > 0.0 ? zscale(1.0 / bt, zconj(tk)) : make_double2(1.0, 0.0);
    alpha[p * n + k] = zmul(sk, ph);
    beta[p * n + k] = make_double2(bt, 0.0);
  }

  // ---- 4. right eigenvectors of (S, T): (beta_k S - alpha_k T) y = 0, y_k = 1, y_i = 0 (i > k)
  for (int k = t; k < n; k += QZ_THREADS) {
    const double2 ak = A[(int64_t)k * n + k], bk = B[(int64_t)k * n + k];
    double2* y = Y + k;   // column k, stride n
    for (int i = n - 1; i > k; --i) y[(int64_t)i * n] = make_double2(0.0, 0.0);
    y[(int64_t)k * n] = make_double2(1.0, 0.0);
    const double small = QZ_EPS * (zabs(ak) * bnorm + zabs(bk) * anorm) + 1e-300;
    for (int i = k - 1; i >= 0; --i) {
      double2 s = make_double2(0.0, 0.0);
      for (int j = i + 1; j <= k; ++j) {
        const double2 c = zsub(zmul(bk, A[(int64_t)i * n + j]), zmul(ak, B[(int64_t)i * n + j]));
        s = zadd(s, zmul(c, y[(int64_t)j * n]));
      }
      double2 d = zsub(zmul(bk, A[(int64_t)i * n + i]), zmul(ak, B[(int64_t)i * n + i]));
      if (zabs(d) < small) d = make_double2(small, 0.0);
      double2 yi = zdiv(make_double2(-s.x, -s.y), d);
      const double m = zabs(yi);
      if (m > 1e100) {   // rescale the vector computed so far
        const double f = 1.0 / m;
        for (int j = i + 1; j <= k; ++j) y[(int64_t)j * n] = zscale(f, y[(int64_t)j * n]);
        yi = zscale(f, yi);
      }
      y[(int64_t)i * n] = yi;
    }
  }
}

// unit 2-norm columns of X (n x n, each column of each matrix of the batch)
__global__ __launch_bounds__(256) void k_normalize_cols(int n, double2* Xall) {
  const int64_t p = blockIdx.y;
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  double2* X = Xall + p * (int64_t)n * n;
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    const double2 v = X[(int64_t)i * n + c];
    s += v.x * v.x + v.y * v.y;
  }
  const double f = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
  for (int i = 0; i < n; ++i) X[(int64_t)i * n + c] = zscale(f, X[(int64_t)i * n + c]);
}

}  // namespace

// Eigenpairs of `batch` n x n pencils (A, B), destroyed (they end as S, T); alpha, beta [batch][n];
// X [batch][n][n] right eigenvectors as unit columns; V, Y scratch [batch][n][n]; status [batch]
ms_status qz_eig(ms_ctx ctx, int n, int batch, double2* A, double2* B, double2* V, double2* Y, double2* alpha,
                 double2* beta, double2* X, int32_t* status) {
  if (n <= 0 || batch <= 0) return MS_OK;
  if (n < 2) return fail(ctx, MS_ERR_UNSUPPORTED, "QZ needs n >= 2");
  const size_t lds = (size_t)n * sizeof(double2);
  if (lds > 64 * 1024) return fail(ctx, MS_ERR_UNSUPPORTED, "QZ pencil size %d > 4096", n);
  {
    Prof prof(ctx, PC_OTHER, 0.0, 0.0);
    hipLaunchKernelGGL(k_qz, dim3(batch), dim3(QZ_THREADS), lds, ctx->stream, n, A, B, V, Y, alpha, beta, status, 30);
    MS_TRY(check_launch(ctx, "qz"));
  }
  GemmArgs g;
  g.M = n; g.N = n; g.K = n;
  g.A = V; g.lda = n; g.sA = (int64_t)n * n;
  g.B = Y; g.ldb = n; g.sB = (int64_t)n * n;
  g.C = X; g.ldc = n; g.sC = (int64_t)n * n;
  g.batch = batch;
  MS_TRY(zgemm(ctx, g));
  hipLaunchKernelGGL(k_normalize_cols, dim3((n + 255) / 256, batch), dim3(256), 0, ctx->stream, n, X);
  return check_launch(ctx, "normalize columns");
}

}  // namespace ms
