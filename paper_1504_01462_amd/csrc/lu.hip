// Batched LU with partial pivoting of an augmented matrix [A | B] and the
// upper-triangular back substitution, complex128.
//
// Right-looking blocked algorithm (two levels: 64-column outer panels made of
// NB-column sub-panels), per sub-panel:
//   1. k_panel:       one workgroup per matrix holds the n x NB panel in
//                     registers, finds each pivot with a wave-shuffle argmax
//                     (|re| + |im|), swaps through LDS and eliminates.
//   2. k_swap_trsm:   one thread per column right of the panel applies the
//                     panel's row interchanges and solves with the unit lower
//                     NB x NB block (rows of U12 and of L^-1 P^T B).
//   3. zgemm:         update of the outer panel's own columns and rows; after
//                     the outer panel, one rank-64 trailing update of the rest
//                     on the matrix cores.
// The right-hand-side columns ride along in steps 2-3, so after the last
// panel they hold L^-1 P^T B and only the back substitution remains:
//   k_trsm_upper:     each workgroup owns 64 right-hand-side columns and walks
//                     the 64-row block rows bottom-up; the off-diagonal part is
//                     an MFMA product over the rows already solved, and the
//                     diagonal block is applied as a product with its inverse
//                     (k_upper_block_inverse, once per matrix and block).
#include <type_traits>

#include "ms_internal.h"

namespace ms {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cinv(double2 a) {
  const double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}

constexpr int PANEL_THREADS = 512;

// compile-time loop: f(std::integral_constant<int, I>) for I in [I0, I1)
template <int I0, int I1, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I0 < I1) {
    f(std::integral_constant<int, I0>{});
    static_for<I0 + 1, I1>(f);
  }
}

__device__ __forceinline__ void set_status(int32_t* status, int64_t idx, int32_t code) {
  if (status) atomicCAS(status + idx, 0, code);
}

// Factor columns [j0, j0+nbp) of rows [j0, n) of each matrix.
template <int RPT, int NB>
__global__ __attribute__((amdgpu_flat_work_group_size(PANEL_THREADS, PANEL_THREADS), amdgpu_waves_per_eu(1, 2))) void k_panel(double2* A, int n, int ld, int64_t strideA, int j0,
                                                          int nbp, int32_t* piv, int32_t* status, int64_t sst) {
  __shared__ double2 prow[NB];
  __shared__ double2 jrow[NB];
  __shared__ double red_v[PANEL_THREADS / 64];
  __shared__ int red_i[PANEL_THREADS / 64];

  const int64_t b = blockIdx.x;
  double2* M = A + b * strideA;
  int32_t* pv = piv + b * (int64_t)n;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;

  double2 a[RPT][NB];
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int r = j0 + t + PANEL_THREADS * s;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      a[s][c] = (r < n && c < nbp) ? M[(int64_t)r * ld + j0 + c] : make_double2(0.0, 0.0);
  }

  static_for<0, NB>([&](auto cidx) {
    constexpr int c = decltype(cidx)::value;
    const int j = j0 + c;
    // local argmax of |re| + |im| over owned rows r >= j
    double bv = -1.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = j0 + t + PANEL_THREADS * s;
      if (r >= j && r < n) {
        const double v = fabs(a[s][c].x) + fabs(a[s][c].y);
        if (v > bv) { bv = v; bi = r; }
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { red_v[wave] = bv; red_i[wave] = bi; }
    __syncthreads();
    bv = red_v[0];
    bi = red_i[0];
#pragma unroll
    for (int w = 1; w < PANEL_THREADS / 64; ++w) {
      const double ov = red_v[w];
      const int oi = red_i[w];
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    const bool active = c < nbp;
    const bool ok = active && (bv > 0.0);
    if (active && !ok && t == 0) {  // zero (or NaN) pivot column: record, leave it as is
      pv[j] = j;
      set_status(status, b * sst, bv == 0.0 ? MS_ERR_SINGULAR : MS_ERR_NONFINITE);
    }
    const int p = ok ? bi : j;
    // rows j and p: owners publish, then exchange
    const int op = p - j0, oj = j - j0;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      if (ok && t + PANEL_THREADS * s == op) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) prow[cc] = a[s][cc];
      }
      if (ok && t + PANEL_THREADS * s == oj) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) jrow[cc] = a[s][cc];
      }
    }
    __syncthreads();
    if (ok) {
      if (p != j) {
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          if (t + PANEL_THREADS * s == oj) {
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) a[s][cc] = prow[cc];
          }
          if (t + PANEL_THREADS * s == op) {
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) a[s][cc] = jrow[cc];
          }
        }
      }
      if (t == 0) pv[j] = p;
      const double2 inv = cinv(prow[c]);
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int r = j0 + t + PANEL_THREADS * s;
        if (r > j && r < n) {
          const double2 l = cmul(a[s][c], inv);
          a[s][c] = l;
#pragma unroll
          for (int cc = c + 1; cc < NB; ++cc) a[s][cc] = csub(a[s][cc], cmul(l, prow[cc]));
        }
      }
    }
    // no barrier here: the next column writes red_v/red_i only after every thread has
    // passed this column's second barrier, and prow/jrow only after its own first one
  });

#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int r = j0 + t + PANEL_THREADS * s;
    if (r < n) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbp) M[(int64_t)r * ld + j0 + c] = a[s][c];
    }
  }
}

// Apply the sub-panel's interchanges to columns [c0, cend) and solve with its unit
// lower block there; columns [s0, s1) (the L columns of the earlier sub-panels of
// the same outer panel) only receive the interchanges.
template <int NB>
__global__ __launch_bounds__(256) void k_swap_trsm(double2* A, int n, int ld, int64_t strideA, int j0, int nbp,
                                                   int c0, int cend, int s0, int s1, const int32_t* piv) {
  __shared__ double2 L[NB][NB];
  __shared__ int sp[NB];
  const int64_t b = blockIdx.y;
  double2* M = A + b * strideA;
  const int t = threadIdx.x;
  for (int idx = t; idx < NB * NB; idx += 256) {
    const int i = idx / NB, k = idx % NB;
    L[i][k] = (i < nbp && k < i) ? M[(int64_t)(j0 + i) * ld + j0 + k] : make_double2(0.0, 0.0);
  }
  if (t < NB) sp[t] = (t < nbp) ? piv[b * (int64_t)n + j0 + t] : 0;
  __syncthreads();
  const int g = blockIdx.x * 256 + t;
  const int nright = cend - c0;
  const bool solve = g < nright;
  const int col = solve ? c0 + g : s0 + (g - nright);
  if (!solve && col >= s1) return;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i < nbp) {
      const int r = j0 + i, p = sp[i];
      double2* pr = M + (int64_t)r * ld + col;
      if (p != r) {
        double2* pp = M + (int64_t)p * ld + col;
        const double2 tmp = *pp;
        *pp = *pr;
        *pr = tmp;
      }
    }
  }
  if (!solve) return;
  double2 x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i < nbp) {
      double2 v = M[(int64_t)(j0 + i) * ld + col];
#pragma unroll
      for (int k = 0; k < NB; ++k)
        if (k < i) v = csub(v, cmul(L[i][k], x[k]));
      x[i] = v;
      M[(int64_t)(j0 + i) * ld + col] = v;
    }
  }
}

// Right of an outer panel [J0, J1): apply its interchanges (in order) to columns
// [c0, ncols) and copy rows [J0, J1) of those columns to T (ldt = ncols - c0).
__global__ __launch_bounds__(256) void k_swap_rows_copy(double2* A, int n, int ld, int64_t strideA, int J0, int J1,
                                                        int c0, int ncols, const int32_t* piv, double2* T,
                                                        int64_t sT) {
  __shared__ int sp[64];
  const int64_t b = blockIdx.y;
  double2* M = A + b * strideA;
  const int t = threadIdx.x;
  if (t < J1 - J0) sp[t] = piv[b * (int64_t)n + J0 + t];
  __syncthreads();
  const int col = c0 + blockIdx.x * 256 + t;
  if (col >= ncols) return;
  for (int i = 0; i < J1 - J0; ++i) {
    const int r = J0 + i, p = sp[i];
    if (p != r) {
      double2* pr = M + (int64_t)r * ld + col;
      double2* pp = M + (int64_t)p * ld + col;
      const double2 tmp = *pp;
      *pp = *pr;
      *pr = tmp;
    }
  }
  double2* Tb = T + b * sT;
  const int ldt = ncols - c0;
  for (int i = 0; i < J1 - J0; ++i) Tb[(int64_t)i * ldt + (col - c0)] = M[(int64_t)(J0 + i) * ld + col];
}

// Inverse of the unit lower triangular m x m block at (J0, J0) (m <= 64), into Linv (ld 64).
__global__ __launch_bounds__(64) void k_unit_lower_inverse(const double2* A, int ld, int64_t strideA, int J0, int m,
                                                           double2* Linv) {
  __shared__ double2 L[64][65];
  __shared__ double2 X[64][65];
  const int64_t b = blockIdx.x;
  const double2* M = A + b * strideA;
  const int t = threadIdx.x;
  for (int idx = t; idx < m * m; idx += 64) {
    const int i = idx / m, k = idx % m;
    L[i][k] = (k < i) ? M[(int64_t)(J0 + i) * ld + J0 + k] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (t < m) {   // column t of L^-1 by forward substitution
    for (int i = 0; i < m; ++i) {
      double2 v = make_double2(i == t ? 1.0 : 0.0, 0.0);
      for (int k = t; k < i; ++k) v = csub(v, cmul(L[i][k], X[k][t]));
      X[i][t] = (i < t) ? make_double2(0.0, 0.0) : v;
    }
  }
  __syncthreads();
  double2* Lb = Linv + b * 64 * 64;
  for (int idx = t; idx < m * m; idx += 64) Lb[(idx / m) * 64 + idx % m] = X[idx / m][idx % m];
}

// Inverses of the 64 x 64 upper triangular diagonal blocks of U (leading n x n of A):
// Dinv[b][ib] (ld 64), one workgroup of 64 threads per block, thread c solves column c.
__global__ __launch_bounds__(64) void k_upper_block_inverse(const double2* A, int n, int ld, int64_t strideA,
                                                           int nblk, double2* Dinv, int32_t* status, int64_t sst) {
  __shared__ double2 D[64][65];
  __shared__ double2 X[64][65];
  const int ib = blockIdx.x;
  const int64_t b = blockIdx.y;
  const double2* M = A + b * strideA;
  const int t = threadIdx.x;
  const int r0 = ib * 64, m = min(64, n - r0);
  for (int idx = t; idx < 64 * 64; idx += 64) {
    const int i = idx / 64, k = idx % 64;
    D[i][k] = (i < m && k < m && k >= i) ? M[(int64_t)(r0 + i) * ld + r0 + k] : make_double2(i == k ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  bool singular = false;
  for (int i = 63; i >= 0; --i) {   // column t of D^-1: D x = e_t, x_i = 0 for i > t
    double2 v = make_double2(i == t ? 1.0 : 0.0, 0.0);
    if (i <= t) {
      for (int k = i + 1; k <= t; ++k) v = csub(v, cmul(D[i][k], X[k][t]));
      const double2 d = D[i][i];
      if (d.x == 0.0 && d.y == 0.0) {
        singular = true;
        v = make_double2(0.0, 0.0);
      } else {
        v = cmul(v, cinv(d));
      }
    } else {
      v = make_double2(0.0, 0.0);
    }
    X[i][t] = v;
  }
  if (singular) set_status(status, b * sst, (int32_t)MS_ERR_SINGULAR);
  __syncthreads();
  double2* Db = Dinv + (b * nblk + ib) * 64 * 64;
  for (int idx = t; idx < 64 * 64; idx += 64) Db[idx] = X[idx / 64][idx % 64];
}

// Back substitution U Y = Z, Z = A[:, n:ncols]: each workgroup owns 64 right-hand-side
// columns (16 per wave) and walks the 64-row block rows bottom-up.  Per block row,
// R = Z_rows - U_rows,below Y_below (MFMA, U staged through LDS in 64 x TR_KC
// chunks, Y read from global), then Y_rows = Dinv R (MFMA, Dinv staged the same way).
constexpr int TR_KC = 32;
__global__ __launch_bounds__(256) void k_trsm_upper(const double2* A, int n, int ld, int64_t strideA, int nrhs,
                                                    const double2* Dinv, int nblk, double2* Y, int64_t ldy,
                                                    int64_t sY) {
  __shared__ double Us[2][64][TR_KC + 1];    // staged U (or Dinv) chunk, re/im
  __shared__ double2 Rs[64][65];             // right-hand sides of the block row
  const int64_t b = blockIdx.y;
  const double2* M = A + b * strideA;
  double2* Yb = Y + b * sY;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int cbase = blockIdx.x * 64;
  const int myc = cbase + wave * 16 + (lane & 15);
  typedef double d4v __attribute__((ext_vector_type(4)));

  for (int ib = nblk - 1; ib >= 0; --ib) {
    const int r0 = ib * 64, r1 = min(n, r0 + 64);
    d4v cr[4], ci[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) { cr[a] = d4v{0, 0, 0, 0}; ci[a] = d4v{0, 0, 0, 0}; }
    // acc = U[r0:r1, r1:n] Y[r1:n, cols]
    for (int k0 = r1; k0 < n; k0 += TR_KC) {
      for (int idx = t; idx < 64 * TR_KC; idx += 256) {
        const int i = idx / TR_KC, k = idx % TR_KC;
        double2 v = make_double2(0.0, 0.0);
        if (r0 + i < r1 && k0 + k < n) v = M[(int64_t)(r0 + i) * ld + k0 + k];
        Us[0][i][k] = v.x;
        Us[1][i][k] = v.y;
      }
      __syncthreads();
      const int kend = min(TR_KC, n - k0);
      for (int kk = 0; kk < kend; kk += 4) {
        const int kl = kk + (lane >> 4);
        double2 y = make_double2(0.0, 0.0);
        if (k0 + kl < n && myc < nrhs) y = Yb[(int64_t)(k0 + kl) * ldy + myc];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const double ar = Us[0][a * 16 + (lane & 15)][kl], ai = Us[1][a * 16 + (lane & 15)][kl];
          cr[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, y.x, cr[a], 0, 0, 0);
          ci[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, y.y, ci[a], 0, 0, 0);
          cr[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, y.y, cr[a], 0, 0, 0);
          ci[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, y.x, ci[a], 0, 0, 0);
        }
      }
      __syncthreads();
    }
    // R = Z - acc
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = a * 16 + (lane >> 4) + 4 * v;   // f64 MFMA accumulator row
        const int r = r0 + i;
        double2 z = make_double2(0.0, 0.0);
        if (r < r1 && myc < nrhs) z = M[(int64_t)r * ld + n + myc];
        Rs[i][wave * 16 + (lane & 15)] = make_double2(z.x - cr[a][v], z.y - ci[a][v]);
      }
#pragma unroll
    for (int a = 0; a < 4; ++a) { cr[a] = d4v{0, 0, 0, 0}; ci[a] = d4v{0, 0, 0, 0}; }
    // Y_rows = Dinv R
    const double2* Di = Dinv + (b * nblk + ib) * 64 * 64;
    for (int k0 = 0; k0 < 64; k0 += TR_KC) {
      __syncthreads();   // Rs complete / previous chunk consumed
      for (int idx = t; idx < 64 * TR_KC; idx += 256) {
        const int i = idx / TR_KC, k = idx % TR_KC;
        const double2 v = Di[i * 64 + k0 + k];
        Us[0][i][k] = v.x;
        Us[1][i][k] = v.y;
      }
      __syncthreads();
      for (int kk = 0; kk < TR_KC; kk += 4) {
        const int kl = kk + (lane >> 4);
        const double2 rr = Rs[k0 + kl][wave * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const double ar = Us[0][a * 16 + (lane & 15)][kl], ai = Us[1][a * 16 + (lane & 15)][kl];
          cr[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, rr.x, cr[a], 0, 0, 0);
          ci[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, rr.y, ci[a], 0, 0, 0);
          cr[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, rr.y, cr[a], 0, 0, 0);
          ci[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, rr.x, ci[a], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + a * 16 + (lane >> 4) + 4 * v;
        if (r < r1 && myc < nrhs) Yb[(int64_t)r * ldy + myc] = make_double2(cr[a][v], ci[a][v]);
      }
    __syncthreads();   // Y rows visible to the whole workgroup; Us/Rs free
  }
}

template <int RPT, int NB>
void launch_panel(ms_ctx ctx, double2* A, int n, int ld, int64_t sA, int batch, int j0, int nbp, int32_t* piv,
                  int32_t* status, int64_t sst) {
  hipLaunchKernelGGL((k_panel<RPT, NB>), dim3(batch), dim3(PANEL_THREADS), 0, ctx->stream, A, n, ld, sA, j0, nbp,
                     piv, status, sst);
}

}  // namespace

namespace {
void trailing(ms_ctx ctx, double2* A, int ncols, int64_t strideA, int batch, int r0, int r1, int c0, int c1, int k0,
              int k1, ms_status* st) {
  if (*st != MS_OK || r1 <= r0 || c1 <= c0 || k1 <= k0) return;
  GemmArgs ga;
  ga.M = r1 - r0;
  ga.N = c1 - c0;
  ga.K = k1 - k0;
  ga.A = A + (int64_t)r0 * ncols + k0;
  ga.lda = ncols;
  ga.sA = strideA;
  ga.B = A + (int64_t)k0 * ncols + c0;
  ga.ldb = ncols;
  ga.sB = strideA;
  ga.C = A + (int64_t)r0 * ncols + c0;
  ga.ldc = ncols;
  ga.sC = strideA;
  ga.alpha = make_double2(-1.0, 0.0);
  ga.beta = make_double2(1.0, 0.0);
  ga.batch = batch;
  ga.prof = PC_LU_UPDATE;
  *st = zgemm(ctx, ga);
}
}  // namespace

// Two-level right-looking LU.  An outer panel [J0, J1) of up to 64 columns is
// factored as sub-panels of nb columns touching only its own columns (panel
// kernel, interchanges + unit-lower solve, update G1 of the outer panel's
// remaining columns).  Then, right of it: all of its interchanges and a copy of
// its rows (k_swap_rows_copy), U12 = L11^-1 B (k_unit_lower_inverse + GEMM) and
// one rank-64 update of the trailing rows (G3).
ms_status getrf_aug(ms_ctx ctx, double2* A, int n, int ncols, int64_t strideA, int batch, int32_t* piv,
                    int32_t* status, int64_t sst) {
  if (n <= 0 || batch <= 0) return MS_OK;
  if (n > 4096) return fail(ctx, MS_ERR_UNSUPPORTED, "LU size %d > 4096", n);
  if (batch > 65535) return fail(ctx, MS_ERR_UNSUPPORTED, "LU batch %d > 65535", batch);
  const int rpt = (n + PANEL_THREADS - 1) / PANEL_THREADS;
  const int nb = rpt <= 3 ? 16 : (rpt <= 6 ? 8 : 4);
  constexpr int OUTER = 64;
  void *tbuf = nullptr, *linv = nullptr;
  const int64_t sT = (int64_t)OUTER * ncols;
  MS_TRY(workspace(ctx, 30, (size_t)batch * sT * sizeof(double2), &tbuf));
  MS_TRY(workspace(ctx, 31, (size_t)batch * OUTER * OUTER * sizeof(double2), &linv));
  ms_status st = MS_OK;
  for (int J0 = 0; J0 < n; J0 += OUTER) {
    const int J1 = std::min(n, J0 + OUTER);
    for (int j0 = J0; j0 < J1; j0 += nb) {
      const int nbp = std::min(nb, J1 - j0);
      {
        Prof prof(ctx, PC_LU_PANEL, 8.0 * nbp * nbp * (double)(n - j0) * batch, 32.0 * nbp * (double)(n - j0) * batch);
        switch (rpt) {
          case 1: launch_panel<1, 16>(ctx, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 2: launch_panel<2, 16>(ctx, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 3: launch_panel<3, 16>(ctx, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 4: launch_panel<4, 8>(ctx, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 5: launch_panel<5, 8>(ctx, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 6: launch_panel<6, 8>(ctx, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 7: launch_panel<7, 4>(ctx, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          default: launch_panel<8, 4>(ctx, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
        }
        MS_TRY(check_launch(ctx, "lu panel"));
      }
      const int c0 = j0 + nbp;
      const int nright = J1 - c0, nleft = j0 - J0;
      if (nright + nleft > 0) {
        dim3 g((nright + nleft + 255) / 256, batch);
        Prof prof(ctx, PC_LU_SWAP, 4.0 * nbp * nbp * (double)nright * batch,
                  64.0 * nbp * (double)(nright + nleft) * batch);
        if (nb == 16)
          hipLaunchKernelGGL((k_swap_trsm<16>), g, dim3(256), 0, ctx->stream, A, n, ncols, strideA, j0, nbp, c0, J1, J0,
                             j0, piv);
        else if (nb == 8)
          hipLaunchKernelGGL((k_swap_trsm<8>), g, dim3(256), 0, ctx->stream, A, n, ncols, strideA, j0, nbp, c0, J1, J0,
                             j0, piv);
        else
          hipLaunchKernelGGL((k_swap_trsm<4>), g, dim3(256), 0, ctx->stream, A, n, ncols, strideA, j0, nbp, c0, J1, J0,
                             j0, piv);
        MS_TRY(check_launch(ctx, "lu swap/trsm"));
      }
      trailing(ctx, A, ncols, strideA, batch, c0, n, c0, J1, j0, c0, &st);   // G1
      MS_TRY(st);
    }
    if (J1 >= ncols) continue;
    const int m = J1 - J0;
    {
      Prof prof(ctx, PC_LU_SWAP, 0.0, 64.0 * m * (double)(ncols - J1) * batch);
      hipLaunchKernelGGL(k_swap_rows_copy, dim3((ncols - J1 + 255) / 256, batch), dim3(256), 0, ctx->stream, A, n,
                         ncols, strideA, J0, J1, J1, ncols, piv, static_cast<double2*>(tbuf), sT);
      MS_TRY(check_launch(ctx, "lu row interchanges"));
      hipLaunchKernelGGL(k_unit_lower_inverse, dim3(batch), dim3(64), 0, ctx->stream, A, ncols, strideA, J0, m,
                         static_cast<double2*>(linv));
      MS_TRY(check_launch(ctx, "lu unit-lower inverse"));
    }
    {  // U12 = L11^-1 B
      GemmArgs ga;
      ga.M = m;
      ga.N = ncols - J1;
      ga.K = m;
      ga.A = linv;
      ga.lda = OUTER;
      ga.sA = OUTER * OUTER;
      ga.B = tbuf;
      ga.ldb = ncols - J1;
      ga.sB = sT;
      ga.C = A + (int64_t)J0 * ncols + J1;
      ga.ldc = ncols;
      ga.sC = strideA;
      ga.batch = batch;
      ga.prof = PC_LU_UPDATE;
      MS_TRY(zgemm(ctx, ga));
    }
    trailing(ctx, A, ncols, strideA, batch, J1, n, J1, ncols, J0, J1, &st);   // G3: rank-64 update
    MS_TRY(st);
  }
  return MS_OK;
}

ms_status trsm_upper_aug(ms_ctx ctx, const double2* A, int n, int ncols, int64_t strideA, int batch, double2* Y,
                         int64_t ldy, int64_t sY, int32_t* status, int64_t sst) {
  const int nrhs = ncols - n;
  if (n <= 0 || nrhs <= 0 || batch <= 0) return MS_OK;
  if (batch > 65535) return fail(ctx, MS_ERR_UNSUPPORTED, "trsm batch %d > 65535", batch);
  const int nblk = (n + 63) / 64;
  void* dinv = nullptr;
  MS_TRY(workspace(ctx, 32, (size_t)batch * nblk * 64 * 64 * sizeof(double2), &dinv));
  Prof prof(ctx, PC_TRSM, 4.0 * (double)n * n * nrhs * batch, 16.0 * batch * ((double)n * n / 2 + 2.0 * n * nrhs));
  hipLaunchKernelGGL(k_upper_block_inverse, dim3(nblk, batch), dim3(64), 0, ctx->stream, A, n, ncols, strideA, nblk,
                     static_cast<double2*>(dinv), status, sst);
  MS_TRY(check_launch(ctx, "upper block inverse"));
  dim3 g((nrhs + 63) / 64, batch);
  hipLaunchKernelGGL(k_trsm_upper, g, dim3(256), 0, ctx->stream, A, n, ncols, strideA, nrhs,
                     static_cast<const double2*>(dinv), nblk, Y, ldy, sY);
  return check_launch(ctx, "trsm upper");
}

}  // namespace ms
