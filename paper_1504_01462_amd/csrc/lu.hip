// Batched LU with partial pivoting of an augmented matrix [A | B] and the
// upper-triangular back substitution, complex128.
//
// Right-looking blocked algorithm (two levels: 128-column outer panels made of
// NB-column sub-panels), per sub-panel:
//   1. k_panel:       one workgroup per matrix holds the n x NB panel in
//                     registers, finds each pivot with a wave-shuffle argmax
//                     (|re| + |im|), swaps through LDS and eliminates.
//   2. k_swap_trsm:   one thread per column right of the panel applies the
//                     panel's row interchanges and solves with the unit lower
//                     NB x NB block (rows of U12 and of L^-1 P^T B).
//   3. zgemm:         update of the outer panel's own columns and rows.
// After an outer panel, right of it: its interchanges composed into one row
// permutation and applied by gathers (k_swap_rows_copy), U12 = L11^-1 B in two
// 64-row halves (k_unit_lower_inverse + zgemm), and one rank-128 trailing
// update of the rest on the matrix cores.
// The right-hand-side columns ride along in steps 2-3, so after the last
// panel they hold L^-1 P^T B and only the back substitution remains:
//   k_trsm_upper:     each workgroup owns 64 right-hand-side columns and walks
//                     the 64-row block rows bottom-up; the off-diagonal part is
//                     an MFMA product over the rows already solved, and the
//                     diagonal block is applied as a product with its inverse
//                     (k_upper_block_inverse, once per matrix and block).
#include <cstdlib>
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

// Pivot search key of row offset r (< 4096) with magnitude v >= 0: the bits of a
// non-negative double order like the value, so the top 51 bits carry v and the low 13
// bits 8191 - r make the smaller row win a tie (magnitudes equal to ~1e-12 relative
// count as ties).  Ineligible rows get key 0, below every eligible key.
__device__ __forceinline__ unsigned long long pivot_key(double v, int r) {
  return ((unsigned long long)__double_as_longlong(v) & ~0x1FFFull) | (unsigned long long)(8191 - r);
}

// max over the 64 lanes of a wave: DPP butterflies inside each row of 16 lanes, then the
// four row results read as scalars
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long k) {
  auto step = [&](auto ctrl) {
    constexpr int C = decltype(ctrl)::value;
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)k, C, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(k >> 32), C, 0xF, 0xF, false);
    const unsigned long long o = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
    k = o > k ? o : k;
  };
  step(std::integral_constant<int, 0xB1>{});    // quad_perm [1,0,3,2]
  step(std::integral_constant<int, 0x4E>{});    // quad_perm [2,3,0,1]
  step(std::integral_constant<int, 0x141>{});   // row_half_mirror
  step(std::integral_constant<int, 0x140>{});   // row_mirror
  unsigned long long m = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)k, 16 * r);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(k >> 32), 16 * r);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    m = o > m ? o : m;
  }
  return m;
}

// Factor columns [j0, j0+nbp) of rows [j0, n) of each matrix.
template <int RPT, int NB>
__global__ __attribute__((amdgpu_flat_work_group_size(PANEL_THREADS, PANEL_THREADS), amdgpu_waves_per_eu(1, 2))) void k_panel(double2* A, int n, int ld, int64_t strideA, int j0,
                                                          int nbp, int32_t* piv, int32_t* status, int64_t sst) {
  __shared__ double2 prow[NB];
  __shared__ double2 jrow[NB];
  __shared__ unsigned long long red_k[PANEL_THREADS / 64];

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
    // argmax of |re| + |im| over rows r >= j: per thread, per wave (DPP), per block (LDS)
    unsigned long long key = 0;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = j0 + t + PANEL_THREADS * s;
      if (r >= j && r < n) {
        const unsigned long long kk = pivot_key(fabs(a[s][c].x) + fabs(a[s][c].y), r - j0);
        key = kk > key ? kk : key;
      }
    }
    key = wave_max_u64(key);
    if (lane == 0) red_k[wave] = key;
    __syncthreads();
    key = red_k[0];
#pragma unroll
    for (int w = 1; w < PANEL_THREADS / 64; ++w) {
      const unsigned long long o = red_k[w];
      key = o > key ? o : key;
    }
    const double bv = __longlong_as_double((long long)(key & ~0x1FFFull));
    const bool active = c < nbp;
    const bool ok = active && key != 0 && bv > 0.0;   // false for a zero or NaN column
    if (active && !ok && t == 0) {  // zero (or NaN) pivot column: record, leave it as is
      pv[j] = j;
      set_status(status, b * sst, (key == 0 || bv == 0.0) ? MS_ERR_SINGULAR : MS_ERR_NONFINITE);
    }
    const int p = ok ? j0 + (8191 - (int)(key & 0x1FFFull)) : j;
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
    // no barrier here: the next column writes red_k only after every thread has
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
// the same outer panel) only receive the interchanges.  The interchanges are
// composed into one permutation of at most 2 NB rows (wave 0), so each column is
// one round of independent loads followed by its stores.
template <int NB>
__global__ __launch_bounds__(256) void k_swap_trsm(double2* A, int n, int ld, int64_t strideA, int j0, int nbp,
                                                   int c0, int cend, int s0, int s1, const int32_t* piv) {
  static_assert(NB <= 64, "one lane per block row");
  __shared__ double2 L[NB][NB];
  __shared__ int s_cont[NB], s_erow[NB], s_esrc[NB];
  __shared__ int s_next;
  const int64_t b = blockIdx.y;
  double2* M = A + b * strideA;
  const int t = threadIdx.x;
  for (int idx = t; idx < NB * NB; idx += 256) {
    const int i = idx / NB, k = idx % NB;
    L[i][k] = (i < nbp && k < i) ? M[(int64_t)(j0 + i) * ld + j0 + k] : make_double2(0.0, 0.0);
  }
  if (t < 64) {
    const int lane = t;
    const int jend = j0 + nbp;
    int cont = j0 + lane;   // original row now held by row j0 + lane
    int erow = -1, esrc = -1;
    int next = 0;
    for (int i = 0; i < nbp; ++i) {
      const int p = piv[b * (int64_t)n + j0 + i];
      const int ci = __shfl(cont, i, 64);
      if (p < jend) {
        const int q = p - j0;
        const int cq = __shfl(cont, q, 64);
        if (lane == i) cont = cq;
        if (lane == q) cont = ci;
      } else {
        const unsigned long long hit = __ballot(lane < next && erow == p);
        if (hit) {
          const int f = __ffsll((long long)hit) - 1;
          const int ef = __shfl(esrc, f, 64);
          if (lane == i) cont = ef;
          if (lane == f) esrc = ci;
        } else {
          if (lane == next) { erow = p; esrc = ci; }
          if (lane == i) cont = p;
          ++next;
        }
      }
    }
    if (lane < NB) {
      s_cont[lane] = cont;
      s_erow[lane] = erow;
      s_esrc[lane] = esrc;
    }
    if (lane == 0) s_next = next;
  }
  __syncthreads();
  const int g = blockIdx.x * 256 + t;
  const int nright = cend - c0;
  const bool solve = g < nright;
  const int col = solve ? c0 + g : s0 + (g - nright);
  if (!solve && col >= s1) return;
  const int ne = s_next;
  double2 x[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) x[k] = M[(int64_t)s_cont[k < nbp ? k : 0] * ld + col];
  if (ne > 0) {   // slots past ne repeat the last row: same value, same address
    double ex[NB], ey[NB];   // (separate planes: a double2 array here ends up in scratch)
#pragma unroll
    for (int f = 0; f < NB; ++f) {
      const double2 v = M[(int64_t)s_esrc[min(f, ne - 1)] * ld + col];
      ex[f] = v.x;
      ey[f] = v.y;
    }
#pragma unroll
    for (int f = 0; f < NB; ++f) M[(int64_t)s_erow[min(f, ne - 1)] * ld + col] = make_double2(ex[f], ey[f]);
  }
  if (solve) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
#pragma unroll
      for (int k = 0; k < i; ++k) x[i] = csub(x[i], cmul(L[i][k], x[k]));
    }
  }
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (k < nbp) M[(int64_t)(j0 + k) * ld + col] = x[k];
}

// Right of an outer panel [J0, J1) (J1 - J0 <= 128): compose its interchanges into
// one row permutation (wave 0, in registers, two rows per lane), then, per column
// in [c0, ncols):
//   T[k]       = row J0+k after the interchanges (k < J1-J0),
//   T[128+f]   = the final content of the f-th row below J1 that the interchanges touch,
// and write those rows back to A.  The rows [J0, J1) of A are not written (the
// U12 product overwrites them).  All loads of a column precede its stores, so
// the gathers are independent instead of a chain of dependent swaps.
constexpr int SWAP_MAX = 128;
__global__ __launch_bounds__(256) void k_swap_rows_copy(double2* A, int n, int ld, int64_t strideA, int J0, int J1,
                                                        int c0, int ncols, const int32_t* piv, double2* T,
                                                        int64_t sT) {
  __shared__ int s_cont[SWAP_MAX], s_erow[SWAP_MAX], s_esrc[SWAP_MAX];
  __shared__ int s_next;
  const int64_t b = blockIdx.y;
  double2* M = A + b * strideA;
  const int t = threadIdx.x;
  const int m = J1 - J0;
  if (t < 64) {
    const int lane = t;
    int cont0 = J0 + lane, cont1 = J0 + 64 + lane;   // original rows now held by rows J0+lane, J0+64+lane
    int erow0 = -1, esrc0 = -1, erow1 = -1, esrc1 = -1;
    int next = 0;                                      // rows >= J1 touched so far (slot next: lane next & 63)
    for (int i = 0; i < m; ++i) {
      const int p = piv[b * (int64_t)n + J0 + i];
      const int ci = __shfl(i < 64 ? cont0 : cont1, i & 63, 64);
      const bool mine_i = lane == (i & 63);
      if (p < J1) {
        const int q = p - J0;
        const int cq = __shfl(q < 64 ? cont0 : cont1, q & 63, 64);
        if (mine_i) { if (i < 64) cont0 = cq; else cont1 = cq; }
        if (lane == (q & 63)) { if (q < 64) cont0 = ci; else cont1 = ci; }
      } else {
        const unsigned long long h0 = __ballot(lane < next && erow0 == p);
        const unsigned long long h1 = __ballot(lane + 64 < next && erow1 == p);
        if (h0 | h1) {
          const int f = h0 ? __ffsll((long long)h0) - 1 : 64 + __ffsll((long long)h1) - 1;
          const int ef = __shfl(f < 64 ? esrc0 : esrc1, f & 63, 64);
          if (mine_i) { if (i < 64) cont0 = ef; else cont1 = ef; }
          if (lane == (f & 63)) { if (f < 64) esrc0 = ci; else esrc1 = ci; }
        } else {
          if (lane == (next & 63)) {
            if (next < 64) { erow0 = p; esrc0 = ci; } else { erow1 = p; esrc1 = ci; }
          }
          if (mine_i) { if (i < 64) cont0 = p; else cont1 = p; }
          ++next;
        }
      }
    }
    s_cont[lane] = cont0;
    s_cont[64 + lane] = cont1;
    s_erow[lane] = erow0;
    s_erow[64 + lane] = erow1;
    s_esrc[lane] = esrc0;
    s_esrc[64 + lane] = esrc1;
    if (lane == 0) s_next = next;
  }
  __syncthreads();
  const int col = c0 + blockIdx.x * 256 + t;
  if (col >= ncols) return;
  const int ne = s_next;
  const int ldt = ncols - c0;
  const int tc = col - c0;
  // A and T never overlap; eight loads are issued before their eight stores
  const double2* __restrict__ src = M + col;
  double2* __restrict__ Tb = T + b * sT + tc;
#define MS_GATHER8(N, IDX, DSTROW, SRCP, SRCROW, DSTP, LDD)                              \
  for (int k0 = 0; k0 < (N); k0 += 8) {                                                 \
    double2 v0, v1, v2, v3, v4, v5, v6, v7;                                             \
    v0 = SRCP[(int64_t)SRCROW(min(k0 + 0, (N) - 1)) * IDX];                             \
    v1 = SRCP[(int64_t)SRCROW(min(k0 + 1, (N) - 1)) * IDX];                             \
    v2 = SRCP[(int64_t)SRCROW(min(k0 + 2, (N) - 1)) * IDX];                             \
    v3 = SRCP[(int64_t)SRCROW(min(k0 + 3, (N) - 1)) * IDX];                             \
    v4 = SRCP[(int64_t)SRCROW(min(k0 + 4, (N) - 1)) * IDX];                             \
    v5 = SRCP[(int64_t)SRCROW(min(k0 + 5, (N) - 1)) * IDX];                             \
    v6 = SRCP[(int64_t)SRCROW(min(k0 + 6, (N) - 1)) * IDX];                             \
    v7 = SRCP[(int64_t)SRCROW(min(k0 + 7, (N) - 1)) * IDX];                             \
    if (k0 + 0 < (N)) DSTP[(int64_t)DSTROW(k0 + 0) * LDD] = v0;                          \
    if (k0 + 1 < (N)) DSTP[(int64_t)DSTROW(k0 + 1) * LDD] = v1;                          \
    if (k0 + 2 < (N)) DSTP[(int64_t)DSTROW(k0 + 2) * LDD] = v2;                          \
    if (k0 + 3 < (N)) DSTP[(int64_t)DSTROW(k0 + 3) * LDD] = v3;                          \
    if (k0 + 4 < (N)) DSTP[(int64_t)DSTROW(k0 + 4) * LDD] = v4;                          \
    if (k0 + 5 < (N)) DSTP[(int64_t)DSTROW(k0 + 5) * LDD] = v5;                          \
    if (k0 + 6 < (N)) DSTP[(int64_t)DSTROW(k0 + 6) * LDD] = v6;                          \
    if (k0 + 7 < (N)) DSTP[(int64_t)DSTROW(k0 + 7) * LDD] = v7;                          \
  }
#define MS_ROW_CONT(k) s_cont[k]
#define MS_ROW_ESRC(k) s_esrc[k]
#define MS_ROW_EROW(k) s_erow[k]
#define MS_ROW_ID(k) (k)
#define MS_ROW_EXT(k) (SWAP_MAX + (k))
  MS_GATHER8(m, ld, MS_ROW_ID, src, MS_ROW_CONT, Tb, ldt)
  MS_GATHER8(ne, ld, MS_ROW_EXT, src, MS_ROW_ESRC, Tb, ldt)
  const double2* __restrict__ Tr = T + b * sT + tc;
  double2* __restrict__ dst = M + col;
  MS_GATHER8(ne, ldt, MS_ROW_EROW, Tr, MS_ROW_EXT, dst, ld)
#undef MS_GATHER8
#undef MS_ROW_CONT
#undef MS_ROW_ESRC
#undef MS_ROW_EROW
#undef MS_ROW_ID
#undef MS_ROW_EXT
}

// Inverse of the unit lower triangular m x m block at (J0, J0) (m <= 64), into Linv
// (ld 64): forward substitution on all 64 unit right-hand sides at once, one
// eliminated row per step; thread (rq, col) owns the rows = rq (mod 4) of column col.
__global__ __launch_bounds__(256) void k_unit_lower_inverse(const double2* A, int ld, int64_t strideA, int J0, int m,
                                                            double2* Linv) {
  __shared__ double2 L[64][65];
  __shared__ double2 X[64][65];
  const int64_t b = blockIdx.x;
  const double2* Mb = A + b * strideA;
  const int t = threadIdx.x;
  for (int idx = t; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, k = idx & 63;
    L[i][k] = (i < m && k < i) ? Mb[(int64_t)(J0 + i) * ld + J0 + k] : make_double2(0.0, 0.0);
    X[i][k] = make_double2(i == k ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int col = t & 63, rq = t >> 6;
  for (int k = 0; k + 1 < m; ++k) {
    const double2 xk = X[k][col];
    for (int i = k + 1 + ((rq - k - 1) & 3); i < m; i += 4) X[i][col] = csub(X[i][col], cmul(L[i][k], xk));
    __syncthreads();
  }
  double2* Lb = Linv + b * 64 * 64;
  for (int idx = t; idx < m * m; idx += 256) Lb[(idx / m) * 64 + idx % m] = X[idx / m][idx % m];
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
// columns and walks the 64-row block rows bottom-up.  Per block row,
// R = Z_rows - U_rows,below Y_below, then Y_rows = Dinv R, both on the matrix cores.
// The 8 waves form two halves that split the K range (alternate TR_KC chunks); within
// a half, wave w owns 16 columns.  U chunks are staged through LDS, one buffer per
// half, and the next chunk of U and of Y is fetched into registers while the current
// one is multiplied.  The halves' partial sums meet in LDS.  Complex products take three
// real MFMAs (Gauss): P1 = Ur Yr, P2 = Ui Yi, P3 = (Ur + Ui)(Yr + Yi), Re = P1 - P2,
// Im = P3 - P1 - P2.
constexpr int TR_KC = 16;
constexpr int TR_THREADS = 512;
__global__ __launch_bounds__(TR_THREADS) void k_trsm_upper(const double2* A, int n, int ld, int64_t strideA,
                                                           int nrhs, const double2* Dinv, int nblk, double2* Y,
                                                           int64_t ldy, int64_t sY) {
  __shared__ double Us[2][2][64][TR_KC + 1];   // [half][re/im][row][k]
  __shared__ double2 Rs[64][65];               // right-hand sides / partial sums of the block row
  typedef double d4v __attribute__((ext_vector_type(4)));
  const int64_t b = blockIdx.y;
  const double2* M = A + b * strideA;
  double2* Yb = Y + b * sY;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int h = wave >> 2, wq = wave & 3, th = t & 255;
  const int cl = wq * 16 + (lane & 15);        // column within the workgroup's 64
  const int myc = blockIdx.x * 64 + cl;
  const bool cok = myc < nrhs;
  constexpr int UE = 64 * TR_KC / 256;         // staged U elements per thread of a half

  for (int ib = nblk - 1; ib >= 0; --ib) {
    const int r0 = ib * 64, r1 = min(n, r0 + 64);
    const int nch = (n - r1 + TR_KC - 1) / TR_KC;   // chunks of the off-diagonal product
    const int iters = (nch + 1) / 2;                 // half h takes chunks h, h+2, ...
    d4v cr[4], ci[4], c3[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) { cr[a] = d4v{0, 0, 0, 0}; ci[a] = d4v{0, 0, 0, 0}; c3[a] = d4v{0, 0, 0, 0}; }
    double2 up[UE], yp[TR_KC / 4];
    // loads with indices clamped into the matrices (no branch, all in flight together);
    // the out-of-range elements are zeroed when the chunk is consumed
    const int mycc = min(myc, nrhs - 1);
    auto fetch = [&](int c) {
      const int k0 = r1 + c * TR_KC;
#pragma unroll
      for (int e = 0; e < UE; ++e) {
        const int idx = th + 256 * e;
        const int i = idx / TR_KC, k = idx % TR_KC;
        up[e] = M[(int64_t)min(r0 + i, r1 - 1) * ld + min(k0 + k, n - 1)];
      }
#pragma unroll
      for (int q = 0; q < TR_KC / 4; ++q) {
        const int k = k0 + 4 * q + (lane >> 4);
        yp[q] = Yb[(int64_t)min(k, n - 1) * ldy + mycc];
      }
    };
    int c = h;
    if (c < nch) fetch(c);
    for (int it = 0; it < iters; ++it, c += 2) {
      const bool have = c < nch;
      double2 yc[TR_KC / 4];
      if (have) {
        const int k0 = r1 + c * TR_KC;
#pragma unroll
        for (int e = 0; e < UE; ++e) {
          const int idx = th + 256 * e;
          const bool ok = r0 + idx / TR_KC < r1 && k0 + idx % TR_KC < n;
          Us[h][0][idx / TR_KC][idx % TR_KC] = ok ? up[e].x : 0.0;
          Us[h][1][idx / TR_KC][idx % TR_KC] = ok ? up[e].y : 0.0;
        }
#pragma unroll
        for (int q = 0; q < TR_KC / 4; ++q) {
          const bool ok = k0 + 4 * q + (lane >> 4) < n && cok;
          yc[q] = ok ? yp[q] : make_double2(0.0, 0.0);
        }
      }
      __syncthreads();
      if (have && c + 2 < nch) fetch(c + 2);
      if (have) {
#pragma unroll
        for (int q = 0; q < TR_KC / 4; ++q) {
          const int kl = 4 * q + (lane >> 4);
          const double ys = yc[q].x + yc[q].y;
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const double ar = Us[h][0][a * 16 + (lane & 15)][kl], ai = Us[h][1][a * 16 + (lane & 15)][kl];
            cr[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, yc[q].x, cr[a], 0, 0, 0);
            ci[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, yc[q].y, ci[a], 0, 0, 0);
            c3[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, ys, c3[a], 0, 0, 0);
          }
        }
      }
      __syncthreads();
    }
    // the halves' partial sums in (re, im) form: cr <- P1 - P2, ci <- P3 - P1 - P2
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double p1 = cr[a][v], p2 = ci[a][v], p3 = c3[a][v];
        cr[a][v] = p1 - p2;
        ci[a][v] = p3 - p1 - p2;
      }
    // R = Z - (partial sum of half 0) - (partial sum of half 1).  Half 0 loads its 16
    // elements of Z (clamped, all in flight together) and writes Z - S0; half 1 then
    // subtracts S1
    if (h == 0) {
      double2 zz[16];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          zz[4 * a + v] = M[(int64_t)min(r0 + a * 16 + (lane >> 4) + 4 * v, r1 - 1) * ld + n + mycc];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = a * 16 + (lane >> 4) + 4 * v;   // f64 MFMA accumulator row
          const double2 z = (r0 + i < r1 && cok) ? zz[4 * a + v] : make_double2(0.0, 0.0);
          Rs[i][cl] = make_double2(z.x - cr[a][v], z.y - ci[a][v]);
        }
    }
    __syncthreads();
    if (h == 1) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = a * 16 + (lane >> 4) + 4 * v;
          const double2 o = Rs[i][cl];
          Rs[i][cl] = make_double2(o.x - cr[a][v], o.y - ci[a][v]);
        }
    }
    __syncthreads();
    // Y_rows = Dinv R; half h takes columns [32 h, 32 h + 32) of Dinv (read from L2)
    const double2* Di = Dinv + (b * nblk + ib) * 64 * 64;
#pragma unroll
    for (int a = 0; a < 4; ++a) { cr[a] = d4v{0, 0, 0, 0}; ci[a] = d4v{0, 0, 0, 0}; c3[a] = d4v{0, 0, 0, 0}; }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kl = 32 * h + 4 * q + (lane >> 4);
      const double2 rr = Rs[kl][cl];
      const double rs = rr.x + rr.y;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const double2 d = Di[(a * 16 + (lane & 15)) * 64 + kl];
        cr[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(d.x, rr.x, cr[a], 0, 0, 0);
        ci[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(d.y, rr.y, ci[a], 0, 0, 0);
        c3[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(d.x + d.y, rs, c3[a], 0, 0, 0);
      }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double p1 = cr[a][v], p2 = ci[a][v], p3 = c3[a][v];
        cr[a][v] = p1 - p2;
        ci[a][v] = p3 - p1 - p2;
      }
    __syncthreads();   // every read of Rs done
    if (h == 1) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) Rs[a * 16 + (lane >> 4) + 4 * v][cl] = make_double2(cr[a][v], ci[a][v]);
    }
    __syncthreads();
    if (h == 0) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = a * 16 + (lane >> 4) + 4 * v;
          const int r = r0 + i;
          const double2 o = Rs[i][cl];
          if (r < r1 && cok) Yb[(int64_t)r * ldy + myc] = make_double2(cr[a][v] + o.x, ci[a][v] + o.y);
        }
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
              int k1, int cat, ms_status* st) {
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
  ga.prof = cat;
  *st = zgemm(ctx, ga);
}
}  // namespace

// workspace of the LU (slots 30, 31) and of the back substitution (slot 32)
static size_t lu_tbuf_bytes(int ncols, int batch) {
  return (size_t)batch * 2 * SWAP_MAX * (size_t)ncols * sizeof(double2);
}
static size_t lu_linv_bytes(int batch) { return (size_t)batch * 64 * 64 * sizeof(double2); }
static size_t trsm_dinv_bytes(int n, int batch) {
  return (size_t)batch * ((n + 63) / 64) * 64 * 64 * sizeof(double2);
}

size_t lu_bytes_per_matrix(int n, int ncols) {
  return lu_tbuf_bytes(ncols, 1) + lu_linv_bytes(1) + trsm_dinv_bytes(n, 1);
}

ms_status lu_reserve(ms_ctx ctx, int n, int ncols, int batch) {
  void* p = nullptr;
  MS_TRY(workspace(ctx, 30, lu_tbuf_bytes(ncols, batch), &p));
  MS_TRY(workspace(ctx, 31, lu_linv_bytes(batch), &p));
  return workspace(ctx, 32, trsm_dinv_bytes(n, batch), &p);
}

// Two-level right-looking LU.  An outer panel [J0, J1) of up to 128 columns is
// factored as sub-panels of nb columns touching only its own columns (panel
// kernel, interchanges + unit-lower solve, update G1 of the outer panel's
// remaining columns).  Then, right of it: all of its interchanges and a copy of
// its rows (k_swap_rows_copy), U12 = L11^-1 B (k_unit_lower_inverse + GEMMs) and
// one rank-128 update of the trailing rows (G3).
ms_status getrf_aug(ms_ctx ctx, double2* A, int n, int ncols, int64_t strideA, int batch, int32_t* piv,
                    int32_t* status, int64_t sst) {
  if (n <= 0 || batch <= 0) return MS_OK;
  if (n > 4096) return fail(ctx, MS_ERR_UNSUPPORTED, "LU size %d > 4096", n);
  if (batch > 65535) return fail(ctx, MS_ERR_UNSUPPORTED, "LU batch %d > 65535", batch);
  const int rpt = (n + PANEL_THREADS - 1) / PANEL_THREADS;
  const int nb = rpt <= 3 ? 16 : (rpt <= 6 ? 8 : 4);
  constexpr int OUTER = SWAP_MAX;   // 128-column outer panels: rank-128 trailing updates
  void *tbuf = nullptr, *linv = nullptr;
  const int64_t sT = (int64_t)2 * OUTER * ncols;   // block rows, then the touched rows below
  MS_TRY(workspace(ctx, 30, lu_tbuf_bytes(ncols, batch), &tbuf));
  MS_TRY(workspace(ctx, 31, lu_linv_bytes(batch), &linv));

  // Look-ahead: the panels are factored on a second stream.  After outer panel k,
  // the main stream first updates only the columns of panel k+1 (G3a), which the
  // panel stream then factors while the main stream updates the rest (G3b).
  ms_ctx cp = ctx;
  bool lookahead = false;
  if (const char* env = getenv("MS_LU_LOOKAHEAD"))
    lookahead = n > OUTER && ncols > n && atoi(env) != 0 && !ctx->capturing && !ctx->arena;
  hipEvent_t ev_panel = nullptr, ev_next = nullptr;
  if (lookahead) {
    MS_TRY(child(ctx, 0, &cp));
    while (ctx->lu_ev.size() < 2) {
      hipEvent_t e = nullptr;
      MS_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      ctx->lu_ev.push_back(e);
    }
    ev_panel = ctx->lu_ev[0];
    ev_next = ctx->lu_ev[1];
    MS_HIP(ctx, hipEventRecord(ev_next, ctx->stream));   // the matrix as built on the main stream
  }

  // factor columns [J0, J1) of rows [J0, n) on context c: sub-panels of nb columns,
  // their interchanges and unit-lower solves, and the update G1 of the remaining
  // columns of [J0, J1)
  auto panel_phase = [&](ms_ctx c, int J0, int J1) -> ms_status {
    ms_status st = MS_OK;
    for (int j0 = J0; j0 < J1; j0 += nb) {
      const int nbp = std::min(nb, J1 - j0);
      {
        Prof prof(c, PC_LU_PANEL, 8.0 * nbp * nbp * (double)(n - j0) * batch, 32.0 * nbp * (double)(n - j0) * batch);
        switch (rpt) {
          case 1: launch_panel<1, 16>(c, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 2: launch_panel<2, 16>(c, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 3: launch_panel<3, 16>(c, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 4: launch_panel<4, 8>(c, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 5: launch_panel<5, 8>(c, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 6: launch_panel<6, 8>(c, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          case 7: launch_panel<7, 4>(c, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
          default: launch_panel<8, 4>(c, A, n, ncols, strideA, batch, j0, nbp, piv, status, sst); break;
        }
        MS_TRY(check_launch(c, "lu panel"));
      }
      const int c0 = j0 + nbp;
      const int nright = J1 - c0, nleft = j0 - J0;
      if (nright + nleft > 0) {
        dim3 g((nright + nleft + 255) / 256, batch);
        Prof prof(c, PC_LU_SWAP, 4.0 * nbp * nbp * (double)nright * batch,
                  64.0 * nbp * (double)(nright + nleft) * batch);
        if (nb == 16)
          hipLaunchKernelGGL((k_swap_trsm<16>), g, dim3(256), 0, c->stream, A, n, ncols, strideA, j0, nbp, c0, J1, J0,
                             j0, piv);
        else if (nb == 8)
          hipLaunchKernelGGL((k_swap_trsm<8>), g, dim3(256), 0, c->stream, A, n, ncols, strideA, j0, nbp, c0, J1, J0,
                             j0, piv);
        else
          hipLaunchKernelGGL((k_swap_trsm<4>), g, dim3(256), 0, c->stream, A, n, ncols, strideA, j0, nbp, c0, J1, J0,
                             j0, piv);
        MS_TRY(check_launch(c, "lu swap/trsm"));
      }
      trailing(c, A, ncols, strideA, batch, c0, n, c0, J1, j0, c0, PC_LU_INNER, &st);   // G1
      MS_TRY(st);
    }
    return MS_OK;
  };

  ms_status st = MS_OK;
  for (int J0 = 0; J0 < n; J0 += OUTER) {
    const int J1 = std::min(n, J0 + OUTER);
    if (lookahead) {
      MS_HIP(ctx, hipStreamWaitEvent(cp->stream, ev_next, 0));
      MS_TRY(panel_phase(cp, J0, J1));
      MS_HIP(ctx, hipEventRecord(ev_panel, cp->stream));
      MS_HIP(ctx, hipStreamWaitEvent(ctx->stream, ev_panel, 0));
    } else {
      MS_TRY(panel_phase(ctx, J0, J1));
    }
    if (J1 >= ncols) continue;
    const int m = J1 - J0;
    const int nr = ncols - J1;
    {
      Prof prof(ctx, PC_LU_SWAP, 0.0, 64.0 * m * (double)nr * batch);
      hipLaunchKernelGGL(k_swap_rows_copy, dim3((nr + 255) / 256, batch), dim3(256), 0, ctx->stream, A, n, ncols,
                         strideA, J0, J1, J1, ncols, piv, static_cast<double2*>(tbuf), sT);
      MS_TRY(check_launch(ctx, "lu row interchanges"));
    }
    // U12 = L11^-1 T in two row halves of at most 64:
    //   U_a = La^-1 T_a,   U_b = Lc^-1 (T_b - Lb U_a),   L11 = [La 0; Lb Lc]
    double2* Tb = static_cast<double2*>(tbuf);
    for (int h0 = 0; h0 < m; h0 += 64) {
      const int mh = std::min(64, m - h0);
      if (h0 > 0) {   // T_b -= Lb U_a
        GemmArgs ga;
        ga.M = mh; ga.N = nr; ga.K = h0;
        ga.A = A + (int64_t)(J0 + h0) * ncols + J0; ga.lda = ncols; ga.sA = strideA;
        ga.B = A + (int64_t)J0 * ncols + J1; ga.ldb = ncols; ga.sB = strideA;
        ga.C = Tb + (int64_t)h0 * nr; ga.ldc = nr; ga.sC = sT;
        ga.alpha = make_double2(-1.0, 0.0);
        ga.beta = make_double2(1.0, 0.0);
        ga.batch = batch;
        ga.prof = PC_LU_INNER;
        MS_TRY(zgemm(ctx, ga));
      }
      {
        Prof prof(ctx, PC_LU_SWAP, 0.0, 0.0);
        hipLaunchKernelGGL(k_unit_lower_inverse, dim3(batch), dim3(256), 0, ctx->stream, A, ncols, strideA, J0 + h0,
                           mh, static_cast<double2*>(linv));
        MS_TRY(check_launch(ctx, "lu unit-lower inverse"));
      }
      GemmArgs ga;
      ga.M = mh; ga.N = nr; ga.K = mh;
      ga.A = linv; ga.lda = 64; ga.sA = 64 * 64;
      ga.B = Tb + (int64_t)h0 * nr; ga.ldb = nr; ga.sB = sT;
      ga.C = A + (int64_t)(J0 + h0) * ncols + J1; ga.ldc = ncols; ga.sC = strideA;
      ga.batch = batch;
      ga.prof = PC_LU_INNER;
      MS_TRY(zgemm(ctx, ga));
    }
    // G3: rank-m update of rows [J1, n), columns [J1, ncols); with look-ahead the
    // columns of the next panel first
    if (J1 < n && lookahead) {
      const int J2 = std::min(n, J1 + OUTER);
      trailing(ctx, A, ncols, strideA, batch, J1, n, J1, J2, J0, J1, PC_LU_UPDATE, &st);   // G3a
      MS_TRY(st);
      MS_HIP(ctx, hipEventRecord(ev_next, ctx->stream));
      trailing(ctx, A, ncols, strideA, batch, J1, n, J2, ncols, J0, J1, PC_LU_UPDATE, &st);   // G3b
    } else {
      trailing(ctx, A, ncols, strideA, batch, J1, n, J1, ncols, J0, J1, PC_LU_UPDATE, &st);
    }
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
  MS_TRY(workspace(ctx, 32, trsm_dinv_bytes(n, batch), &dinv));
  Prof prof(ctx, PC_TRSM, 4.0 * (double)n * n * nrhs * batch, 16.0 * batch * ((double)n * n / 2 + 2.0 * n * nrhs));
  hipLaunchKernelGGL(k_upper_block_inverse, dim3(nblk, batch), dim3(64), 0, ctx->stream, A, n, ncols, strideA, nblk,
                     static_cast<double2*>(dinv), status, sst);
  MS_TRY(check_launch(ctx, "upper block inverse"));
  dim3 g((nrhs + 63) / 64, batch);
  hipLaunchKernelGGL(k_trsm_upper, g, dim3(TR_THREADS), 0, ctx->stream, A, n, ncols, strideA, nrhs,
                     static_cast<const double2*>(dinv), nblk, Y, ldy, sY);
  return check_launch(ctx, "trsm upper");
}

}  // namespace ms
