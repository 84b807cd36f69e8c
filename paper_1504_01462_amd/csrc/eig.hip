// E-independent stage: slice Hamiltonians (Sec. II.A, Eq. loc), their
// eigenpairs, and the interface overlaps O^p = U^p^dagger U^{p+1} (App. A).
//
// Eigensolver: one-sided block Jacobi (Hestenes) on the shifted, positive
// definite A = H + c I.  Columns are grouped in blocks of 16; a sweep visits
// every pair of blocks once in round-robin order (nb-1 rounds of nb/2
// disjoint pairs, one launch per round, one workgroup per pair and matrix).
// For a pair, P = W[:, I u J] (n x 32):
//   G = P^dagger P       Gram on the matrix cores (k split over the 4 waves)
//   G = Q diag Q^dagger  cyclic Jacobi on the 32 x 32 Hermitian G in LDS
//   P <- P Q             on the matrix cores, rows staged through LDS
// which makes the 32 columns mutually orthogonal.  At convergence
// W = A V has orthogonal columns; since A is Hermitian positive definite its
// eigenvectors are the normalised columns u_j = w_j / |w_j| and its
// eigenvalues |w_j| - c.  The eigenvalues returned are the Rayleigh quotients
// u_j^dagger H u_j (one extra GEMM), whose error is second order in the
// eigenvector error.  Pairs already orthogonal to the tolerance are skipped; a
// matrix whose previous sweep rotated nothing exits at once.
#include "ms_internal.h"

namespace ms {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// ---- kinetic energies and lead channel energies ---------------------------------------
__global__ void k_kin_eps(int n, const int32_t* g, double b1x, double b1y, double b2x, double b2y, double kx,
                          double ky, double vl, double vr, double* kin, double* el, double* er) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double m1 = g[2 * i], m2 = g[2 * i + 1];
  const double x = kx + m1 * b1x + m2 * b2x, y = ky + m1 * b1y + m2 * b2y;
  const double q = x * x + y * y;
  kin[i] = q;
  el[i] = q + vl;
  er[i] = q + vr;
}

// ---- positivity shift per slice --------------------------------------------------------
// lambda_min(H^p) >= min_i |k+G_i|^2 + V^p(0) - sum_{Q != 0} |V^p(Q)|  (Gershgorin, every
// difference vector appears at most once per row); c = max(0, -bound) + 1.
__global__ __launch_bounds__(256) void k_shift(int n, const double* kin, int64_t n_q, int64_t vstride,
                                               const double2* vq, int q0, double* shift) {
  __shared__ double s_min[256], s_sum[256];
  const int b = blockIdx.x, t = threadIdx.x;
  const double2* v = vq + (int64_t)b * vstride;
  double mn = 1e300, sm = 0.0;
  for (int i = t; i < n; i += 256) mn = fmin(mn, kin[i]);
  for (int64_t q = t; q < n_q; q += 256)
    if (q != q0) sm += sqrt(v[q].x * v[q].x + v[q].y * v[q].y);
  s_min[t] = mn;
  s_sum[t] = sm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      s_min[t] = fmin(s_min[t], s_min[t + o]);
      s_sum[t] += s_sum[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double bound = s_min[0] + v[q0].x - s_sum[0];
    shift[b] = fmax(0.0, -bound) + 1.0;
  }
}

// ---- W = H^p + c_p I --------------------------------------------------------------------
__global__ void k_hgather(int n, const double* kin, const double* shift, int64_t vstride, const double2* vq,
                          const int32_t* q_of_ij, double2* W) {
  const int64_t b = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  double2 h = vq[b * vstride + q_of_ij[idx]];
  if (i == j) h.x += kin[i] + (shift ? shift[b] : 0.0);
  W[b * (int64_t)n * n + idx] = h;
}

// ---- one round of the block Jacobi sweep -----------------------------------------------
constexpr int BW = 16;     // block width
constexpr int PW = 32;     // pair width
constexpr int ROWS = 64;   // rows staged per update step
// Inner sweeps per pair visit.  The pair's columns are rotated again on later visits, so its
// Gram matrix need not be diagonal to full precision after each one: two sweeps (quadratic
// convergence from a nearly diagonal Gram in the later outer sweeps) took 10 % less time than
// sweeping to convergence (up to 12) on config3 slices, with the same eigenvalues and
// residuals; the outer sweeps still run until no pair exceeds the tolerance.
constexpr int INNER_SWEEPS = 2;

struct JacobiArgs {
  double2* W;
  int n;
  int nb_real;             // number of real column blocks
  const int2* pairs;       // this round's pairs
  int32_t* counter;        // [batch][max_sweeps] rotations per sweep
  int max_sweeps;
  int sweep;
  double tol;              // relative off-diagonal tolerance
  // skip record: stamp (sweep x rounds + round) at which each column block was last rotated,
  // [batch][nblk], and at which each pair was last found orthogonal, [batch][rounds x per]
  // (-1: never); a pair whose blocks have not been rotated since it was found orthogonal has
  // the same Gram matrix and is skipped without reading its columns
  int32_t* bmod;
  int32_t* pconv;
  int nblk, npairs, round, per;
};

__device__ __forceinline__ int pair_col(int a, int I, int J, int mI, int mJ) {
  // local column a (0..31) -> global column, or -1 for padding
  if (a < BW) return a < mI ? I * BW + a : -1;
  return (a - BW) < mJ ? J * BW + (a - BW) : -1;
}

__global__ __launch_bounds__(256) void k_jacobi_round(JacobiArgs args) {
  // Gb: the pair's Gram matrix in two buffers (the inner Jacobi reads one and writes the
  // other); the row staging of the P update reuses the same bytes afterwards
  __shared__ __align__(16) double2 Gb[2][PW][PW + 1];
  __shared__ double2 Q[PW][PW + 1];
  __shared__ int s_flag;
  double2(*G)[PW + 1] = Gb[0];
  double(*Ps)[ROWS][PW] = reinterpret_cast<double(*)[ROWS][PW]>(&Gb[0][0][0]);
  static_assert(sizeof(double) * 2 * ROWS * PW <= sizeof(double2) * 2 * PW * (PW + 1), "P staging fits Gb");

  const int64_t b = blockIdx.y;
  // the wave index is uniform across the wave: keeping it scalar keeps the per-wave row
  // loops below scalar loops (no exec-masked divergence around the MFMAs)
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  int32_t* cnt = args.counter + b * args.max_sweeps;
  if (args.sweep > 0 && cnt[args.sweep - 1] == 0) return;  // converged in the previous sweep
  const int n = args.n;
  const int2 pr = args.pairs[blockIdx.x];
  const int I = pr.x, J = pr.y;
  const int mI = (I < args.nb_real) ? min(BW, n - I * BW) : 0;
  const int mJ = (J < args.nb_real) ? min(BW, n - J * BW) : 0;
  if (mI + mJ == 0) return;
  double2* W = args.W + b * (int64_t)n * n;
  const int stamp = args.sweep * (args.nblk - 1) + args.round;
  int32_t* bmod = args.bmod + b * args.nblk;
  int32_t* pconv = args.pconv + b * args.npairs + args.round * args.per + blockIdx.x;
  {
    const int cst = *pconv;
    if (cst >= 0 && bmod[I] < cst && bmod[J] < cst) return;   // unchanged since found orthogonal
  }

  // Columns of the pair are read with indices clamped into this workgroup's own columns
  // (padding lanes read a real column of the pair and discard it), so every load is
  // unconditional and the next rows' loads can be in flight while the MFMAs run.
  const int own0 = (mI > 0) ? I * BW : J * BW;

  // --- Gram G = P^dagger P: each wave takes a quarter of the rows for all three blocks
  {
    d4_t g00r = {0, 0, 0, 0}, g00i = {0, 0, 0, 0}, g01r = {0, 0, 0, 0}, g01i = {0, 0, 0, 0},
         g11r = {0, 0, 0, 0}, g11i = {0, 0, 0, 0}, g003 = {0, 0, 0, 0}, g013 = {0, 0, 0, 0}, g113 = {0, 0, 0, 0};
    const int c = lane & 15;
    const bool okI = c < mI, okJ = c < mJ;
    const int colI = okI ? I * BW + c : own0;
    const int colJ = okJ ? J * BW + c : own0;
    const int kq = (n + 3) / 4;                 // rows per wave, rounded to steps of 4
    const int kbeg = wave * ((kq + 3) / 4 * 4);
    const int kend = min(n, kbeg + (kq + 3) / 4 * 4);
    constexpr int GS = 4;                       // steps of 4 rows per group
    double2 xi[GS], xj[GS], yi[GS], yj[GS];
    auto fetch = [&](int k0, double2* vi, double2* vj) {
#pragma unroll
      for (int s = 0; s < GS; ++s) {
        const int64_t k = min(k0 + 4 * s + (lane >> 4), n - 1);
        vi[s] = W[k * n + colI];
        vj[s] = W[k * n + colJ];
      }
    };
    if (kbeg < kend) fetch(kbeg, xi, xj);
    for (int k0 = kbeg; k0 < kend; k0 += 4 * GS) {
      if (k0 + 4 * GS < kend) fetch(k0 + 4 * GS, yi, yj);
#pragma unroll
      for (int s = 0; s < GS; ++s) {
        const bool okk = k0 + 4 * s + (lane >> 4) < kend;
        const double2 pi = (okk && okI) ? xi[s] : make_double2(0.0, 0.0);
        const double2 pj = (okk && okJ) ? xj[s] : make_double2(0.0, 0.0);
        // A = conj(P_X)^T (16 x 4), B = P_Y (4 x 16): lane holds element (c, k) of both.  Three
        // real products per block (Gauss): P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi) with
        // Ar = Re P_X, Ai = -Im P_X; Re G = P1 - P2, Im G = P3 - P1 - P2 (combined in the reduction)
        const double di = pi.x - pi.y, sj = pj.x + pj.y, si = pi.x + pi.y;
        g00r = __builtin_amdgcn_mfma_f64_16x16x4f64(pi.x, pi.x, g00r, 0, 0, 0);
        g00i = __builtin_amdgcn_mfma_f64_16x16x4f64(-pi.y, pi.y, g00i, 0, 0, 0);
        g003 = __builtin_amdgcn_mfma_f64_16x16x4f64(di, si, g003, 0, 0, 0);
        g01r = __builtin_amdgcn_mfma_f64_16x16x4f64(pi.x, pj.x, g01r, 0, 0, 0);
        g01i = __builtin_amdgcn_mfma_f64_16x16x4f64(-pi.y, pj.y, g01i, 0, 0, 0);
        g013 = __builtin_amdgcn_mfma_f64_16x16x4f64(di, sj, g013, 0, 0, 0);
        g11r = __builtin_amdgcn_mfma_f64_16x16x4f64(pj.x, pj.x, g11r, 0, 0, 0);
        g11i = __builtin_amdgcn_mfma_f64_16x16x4f64(-pj.y, pj.y, g11i, 0, 0, 0);
        g113 = __builtin_amdgcn_mfma_f64_16x16x4f64(pj.x - pj.y, sj, g113, 0, 0, 0);
      }
#pragma unroll
      for (int s = 0; s < GS; ++s) {
        xi[s] = yi[s];
        xj[s] = yj[s];
      }
    }
    // reduce the four partial Grams through LDS (G then Q used as scratch)
    for (int idx = t; idx < PW * PW; idx += 256) G[idx / PW][idx % PW] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int w = 0; w < 4; ++w) {
      if (wave == w) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = (lane >> 4) + 4 * v, j = lane & 15;   // f64 MFMA accumulator layout
          G[i][j] = cadd(G[i][j], make_double2(g00r[v] - g00i[v], g003[v] - g00r[v] - g00i[v]));
          G[i][BW + j] = cadd(G[i][BW + j], make_double2(g01r[v] - g01i[v], g013[v] - g01r[v] - g01i[v]));
          G[BW + i][BW + j] = cadd(G[BW + i][BW + j], make_double2(g11r[v] - g11i[v], g113[v] - g11r[v] - g11i[v]));
        }
      }
      __syncthreads();
    }
    for (int idx = t; idx < BW * BW; idx += 256) {
      const int i = idx / BW, j = idx % BW;
      G[BW + j][i] = cconj(G[i][BW + j]);
    }
    if (t == 0) s_flag = 0;
    __syncthreads();
  }

  // --- convergence test of the pair
  {
    bool rot = false;
    for (int idx = t; idx < PW * PW; idx += 256) {
      const int a = idx / PW, c = idx % PW;
      if (a < c) {
        const double gaa = G[a][a].x, gcc = G[c][c].x;
        const double g2 = G[a][c].x * G[a][c].x + G[a][c].y * G[a][c].y;
        if (gaa > 0.0 && gcc > 0.0 && g2 > args.tol * args.tol * gaa * gcc) rot = true;
      }
    }
    if (rot) s_flag = 1;
    __syncthreads();
    if (s_flag == 0) {
      if (t == 0) *pconv = stamp;
      return;
    }
    if (t == 0) {
      atomicAdd(cnt + args.sweep, 1);
      *pconv = -1;
      bmod[I] = stamp;   // written before the rotated columns, read only by later launches
      bmod[J] = stamp;
    }
  }

  // --- cyclic Jacobi on G (32 x 32 Hermitian), Q accumulates the rotations.  A round applies
  //     16 disjoint rotations (circle-method pairs).  Lane l of every wave forms rotation l % 16
  //     from the current buffer and the lanes exchange them by wave shuffles; thread t owns the
  //     2 x 2 block of G at (row pair t / 16, column pair t % 16) and rows t / 16, t / 16 + 16
  //     of Q in that column pair, and writes its block into the other buffer, so a round needs
  //     one barrier.  Rows then columns, as G' = R^dagger G R:
  //       rows:    G'_a = c G_a - s e^{i phi} G_b ;  G'_b = s e^{-i phi} G_a + c G_b
  //       columns: X'_a = c X_a - s e^{-i phi} X_b ;  X'_b = s e^{i phi} X_a + c X_b
  //     with e^{i phi} = G_ab / |G_ab|, t = sign(z) / (|z| + sqrt(1 + z^2)), z = (G_bb - G_aa) /
  //     (2 |G_ab|), c = 1 / sqrt(1 + t^2), s = t c.  Q's columns drift from unitarity only by
  //     rounding; the Newton-Schulz step below restores it.
  for (int idx = t; idx < PW * PW; idx += 256) {
    const int a = idx / PW, c = idx % PW;
    Q[a][c] = make_double2(a == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();   // every thread has read the pair's flag above before it is reset
  if (t == 0) s_flag = 0;
  __syncthreads();
  int cur = 0;
  {
    const int kr = t >> 4, kc = t & 15, kl = lane & 15;
    auto ends = [](int k, int r, int* lo, int* hi) {
      const int a = (k == 0) ? 0 : ((k - 1 + r) % (PW - 1)) + 1;
      const int c = ((PW - 1 - k - 1 + r) % (PW - 1)) + 1;
      *lo = min(a, c);
      *hi = max(a, c);
    };
    for (int sw = 0; sw < INNER_SWEEPS; ++sw) {
      for (int r = 0; r < PW - 1; ++r) {
        const double2(*Gc)[PW + 1] = Gb[cur];
        double2(*Gn)[PW + 1] = Gb[cur ^ 1];
        // this lane's rotation kl
        int lo, hi;
        ends(kl, r, &lo, &hi);
        double cs = 1.0, sn = 0.0, px = 1.0, py = 0.0;
        {
          const double al = Gc[lo][lo].x, ga = Gc[hi][hi].x;
          const double2 be = Gc[lo][hi];
          const double m2 = be.x * be.x + be.y * be.y, aga = fabs(al * ga);
          if (m2 > 1e-34 * aga && m2 > 0.0) {
            const double inv = rsqrt(m2);
            const double zeta = 0.5 * (ga - al) * inv;
            const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            cs = rsqrt(1.0 + tt * tt);
            sn = tt * cs;
            px = be.x * inv;
            py = be.y * inv;
            if (wave == 0 && lane < 16 && m2 > 1e-30 * aga) s_flag = 1;
          }
        }
        // row rotation kr and column rotation kc from the lanes that formed them
        const double rcs = __shfl(cs, kr), rsn = __shfl(sn, kr), rpx = __shfl(px, kr), rpy = __shfl(py, kr);
        const double ccs = __shfl(cs, kc), csn = __shfl(sn, kc), cpx = __shfl(px, kc), cpy = __shfl(py, kc);
        int rlo, rhi, clo, chi;
        ends(kr, r, &rlo, &rhi);
        ends(kc, r, &clo, &chi);
        const double2 rph = make_double2(rpx, rpy), cph = make_double2(cpx, cpy);
        const int cols[2] = {clo, chi}, rows[2] = {rlo, rhi};
        double2 x[2][2];
#pragma unroll
        for (int v = 0; v < 2; ++v) {        // row rotation of the block's two columns
          const double2 ga = Gc[rlo][cols[v]], gb = Gc[rhi][cols[v]];
          x[0][v] = cadd(cscale(rcs, ga), cscale(-rsn, cmul(rph, gb)));
          x[1][v] = cadd(cscale(rsn, cmul(cconj(rph), ga)), cscale(rcs, gb));
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {        // column rotation of the rotated rows
          const double2 xa = x[u][0], xb = x[u][1];
          Gn[rows[u]][clo] = cadd(cscale(ccs, xa), cscale(-csn, cmul(cconj(cph), xb)));
          Gn[rows[u]][chi] = cadd(cscale(csn, cmul(cph, xa)), cscale(ccs, xb));
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {        // Q <- Q R on rows kr, kr + 16 (in place: own elements)
          const int q = kr + 16 * u;
          const double2 xa = Q[q][clo], xb = Q[q][chi];
          Q[q][clo] = cadd(cscale(ccs, xa), cscale(-csn, cmul(cconj(cph), xb)));
          Q[q][chi] = cadd(cscale(csn, cmul(cph, xa)), cscale(ccs, xb));
        }
        cur ^= 1;
        __syncthreads();
      }
      // every thread reads the flag before thread 0 may reset it for the next sweep
      const bool rotated = s_flag != 0;
      __syncthreads();
      if (!rotated) break;
      if (t == 0) s_flag = 0;
      __syncthreads();
    }
  }
  (void)cur;

  // --- Q <- Q (3 I - Q^dagger Q) / 2: one Newton-Schulz step restores unitarity to
  //     O(|Q^dagger Q - I|^2), so repeated pair updates do not drift the column norms
  {
    double2(*Qn)[PW + 1] = Gb[1];
    for (int idx = t; idx < PW * PW; idx += 256) {      // G <- Q^dagger Q
      const int a = idx / PW, c = idx % PW;
      double2 acc = make_double2(0.0, 0.0);
      for (int k = 0; k < PW; ++k) acc = cadd(acc, cmul(cconj(Q[k][a]), Q[k][c]));
      G[a][c] = acc;
    }
    __syncthreads();
    for (int idx = t; idx < PW * PW; idx += 256) {      // G <- (3 I - G) / 2
      const int a = idx / PW, c = idx % PW;
      const double2 g = G[a][c];
      G[a][c] = make_double2((a == c ? 1.5 : 0.0) - 0.5 * g.x, -0.5 * g.y);
    }
    __syncthreads();
    for (int idx = t; idx < PW * PW; idx += 256) {      // Qn <- Q G
      const int a = idx / PW, c = idx % PW;
      double2 acc = make_double2(0.0, 0.0);
      for (int k = 0; k < PW; ++k) acc = cadd(acc, cmul(Q[a][k], G[k][c]));
      Qn[a][c] = acc;
    }
    __syncthreads();
    for (int idx = t; idx < PW * PW; idx += 256) Q[idx / PW][idx % PW] = Qn[idx / PW][idx % PW];
    __syncthreads();
  }

  // --- P <- P Q, ROWS rows at a time; waves split the 64 x 32 output into 16-row slabs.
  //     The next chunk's loads are issued before the current chunk's MFMAs (rows clamped,
  //     never into the chunk being written: only issued while r0 + ROWS < n).
  constexpr int EP = ROWS * PW / 256;
  double2 pv[EP];
  auto pload = [&](int r0) {
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      const int idx = t + 256 * e;
      const int i = idx / PW, a = idx % PW;
      const int col = pair_col(a, I, J, mI, mJ);
      const int64_t row = min(r0 + i, n - 1);
      pv[e] = W[row * n + (col >= 0 ? col : own0)];
    }
  };
  pload(0);
  for (int r0 = 0; r0 < n; r0 += ROWS) {
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      const int idx = t + 256 * e;
      const int i = idx / PW, a = idx % PW;
      const bool ok = r0 + i < n && pair_col(a, I, J, mI, mJ) >= 0;
      Ps[0][i][a] = ok ? pv[e].x : 0.0;
      Ps[1][i][a] = ok ? pv[e].y : 0.0;
    }
    __syncthreads();
    if (r0 + ROWS < n) pload(r0 + ROWS);
    // three real products per complex block: P1 = Pr Qr, P2 = Pi Qi, P3 = (Pr + Pi)(Qr + Qi)
    d4_t a0 = {0, 0, 0, 0}, b0 = {0, 0, 0, 0}, c0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0}, b1 = {0, 0, 0, 0},
         c1 = {0, 0, 0, 0};
    const int rr = wave * 16;
#pragma unroll
    for (int kk = 0; kk < PW; kk += 4) {
      const int k = kk + (lane >> 4);
      const double ar = Ps[0][rr + (lane & 15)][k], ai = Ps[1][rr + (lane & 15)][k];
      const double2 q0 = Q[k][lane & 15], q1 = Q[k][16 + (lane & 15)];
      const double as = ar + ai;
      a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, q0.x, a0, 0, 0, 0);
      b0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, q0.y, b0, 0, 0, 0);
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(as, q0.x + q0.y, c0, 0, 0, 0);
      a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, q1.x, a1, 0, 0, 0);
      b1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, q1.y, b1, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(as, q1.x + q1.y, c1, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + rr + (lane >> 4) + 4 * v;
      if (row < n) {
        const int col0 = pair_col(lane & 15, I, J, mI, mJ);
        const int col1 = pair_col(16 + (lane & 15), I, J, mI, mJ);
        if (col0 >= 0) W[(int64_t)row * n + col0] = make_double2(a0[v] - b0[v], c0[v] - a0[v] - b0[v]);
        if (col1 >= 0) W[(int64_t)row * n + col1] = make_double2(a1[v] - b1[v], c1[v] - a1[v] - b1[v]);
      }
    }
    __syncthreads();
  }
}

// ---- normalise the converged columns in place: w_j <- w_j / |w_j| ---------------------------
__global__ __launch_bounds__(256) void k_jacobi_normalize(double2* Wall, int n, const int32_t* counter, int max_sweeps,
                                                          int32_t* status) {
  const int64_t b = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  double2* W = Wall + b * (int64_t)n * n;
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    const double2 w = W[(int64_t)i * n + j];
    s += w.x * w.x + w.y * w.y;
  }
  const double inv = 1.0 / sqrt(s);
  for (int i = 0; i < n; ++i) {
    const double2 w = W[(int64_t)i * n + j];
    W[(int64_t)i * n + j] = make_double2(w.x * inv, w.y * inv);
  }
  if (j == 0 && status && counter[b * max_sweeps + max_sweeps - 1] != 0) atomicCAS(status, 0, (int32_t)MS_ERR_NOCONV);
}

// ---- Rayleigh quotients lambda_j = Re(u_j^dagger (H u_j)), sort ascending, emit eigenpairs ----
__global__ __launch_bounds__(256) void k_jacobi_emit(const double2* Wall, const double2* Zall, int n, double* eps_out,
                                                     int64_t eps_stride, double2* Uall, int64_t u_stride) {
  extern __shared__ double sh[];
  double* lam = sh;                  // [n]
  int* rank = (int*)(sh + n);        // [n]
  const int64_t b = blockIdx.x;
  const int t = threadIdx.x;
  const double2* W = Wall + b * (int64_t)n * n;
  const double2* Z = Zall + b * (int64_t)n * n;
  double2* U = Uall + b * u_stride;
  for (int j = t; j < n; j += 256) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      const double2 w = W[(int64_t)i * n + j], z = Z[(int64_t)i * n + j];
      s += w.x * z.x + w.y * z.y;
    }
    lam[j] = s;
  }
  __syncthreads();
  for (int j = t; j < n; j += 256) {
    int r = 0;
    const double lj = lam[j];
    for (int i = 0; i < n; ++i) r += (lam[i] < lj) || (lam[i] == lj && i < j);
    rank[j] = r;
    eps_out[b * eps_stride + r] = lj;
  }
  __syncthreads();
  for (int j = t; j < n; j += 256) {
    const int r = rank[j];
    for (int i = 0; i < n; ++i) U[(int64_t)i * n + r] = W[(int64_t)i * n + j];
  }
}

// min and max of an int32 array (one workgroup)
__global__ __launch_bounds__(256) void k_minmax(int64_t count, const int32_t* v, int32_t* out) {
  __shared__ int smin[256], smax[256];
  const int t = threadIdx.x;
  int mn = 0x7fffffff, mx = -0x7fffffff - 1;
  for (int64_t i = t; i < count; i += 256) {
    mn = min(mn, v[i]);
    mx = max(mx, v[i]);
  }
  smin[t] = mn;
  smax[t] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      smin[t] = min(smin[t], smin[t + o]);
      smax[t] = max(smax[t], smax[t + o]);
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = smin[0];
    out[1] = smax[0];
  }
}

// O = U (copy) or O = U^dagger
__global__ void k_copy_overlap(int n, const double2* U, double2* O, int conj_transpose) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  O[idx] = conj_transpose ? cconj(U[(int64_t)j * n + i]) : U[idx];
}

}  // namespace

ms_status launch_kin_eps(ms_ctx ctx, int n, const int32_t* g_mn, const double* bvec, const double* kpar, double vl,
                         double vr, double* kin, double* eps_left, double* eps_right) {
  hipLaunchKernelGGL(k_kin_eps, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, g_mn, bvec[0], bvec[1], bvec[2],
                     bvec[3], kpar[0], kpar[1], vl, vr, kin, eps_left, eps_right);
  return check_launch(ctx, "kin/eps");
}

ms_status launch_slice_shift(ms_ctx ctx, int n, int nb, const double* kin, int64_t n_q, int64_t vstride,
                             const double2* vq, int q0, double* shift) {
  hipLaunchKernelGGL(k_shift, dim3(nb), dim3(256), 0, ctx->stream, n, kin, n_q, vstride, vq, q0, shift);
  return check_launch(ctx, "shift");
}

ms_status launch_hgather(ms_ctx ctx, int n, int nb, const double* kin, const double* shift, int64_t vstride,
                         const double2* vq, const int32_t* q_of_ij, double2* W) {
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(k_hgather, dim3((unsigned)((nn + 255) / 256), nb), dim3(256), 0, ctx->stream, n, kin, shift,
                     vstride, vq, q_of_ij, W);
  return check_launch(ctx, "hgather");
}

// Z[i] = Uref[r(i)], r(i) = the reference slice nearest to slice s0 + i (references at
// multiples of stride, nref of them)
__global__ void k_gather_ref(int64_t nn, int s0, int stride, int nref, const double2* Uref, double2* Z) {
  const int64_t i = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  const int r = min(nref - 1, (int)((s0 + i + stride / 2) / stride));
  Z[i * nn + idx] = Uref[(int64_t)r * nn + idx];
}

ms_status launch_gather_ref(ms_ctx ctx, int n, int nb, int s0, int stride, int nref, const double2* Uref,
                            double2* Z) {
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(k_gather_ref, dim3((unsigned)((nn + 255) / 256), nb), dim3(256), 0, ctx->stream, nn, s0, stride,
                     nref, Uref, Z);
  return check_launch(ctx, "gather reference eigenvectors");
}

ms_status jacobi_eigh(ms_ctx ctx, int n, int nb, double2* W, const double2* H, double2* Z, double* eps_out,
                      int64_t eps_stride, double2* U, int64_t u_stride, int32_t* status) {
  const int nb_real = (n + BW - 1) / BW;
  const int nblk = nb_real + (nb_real & 1);
  const int rounds = nblk - 1, per = nblk / 2;
  const int max_sweeps = 24;
  // round-robin schedule (circle method), built on the host
  std::vector<int2> pairs((size_t)std::max(rounds, 1) * per);
  for (int r = 0; r < rounds; ++r)
    for (int k = 0; k < per; ++k) {
      const int a = (k == 0) ? 0 : ((k - 1 + r) % (nblk - 1)) + 1;
      const int c = ((nblk - 1 - k - 1 + r) % (nblk - 1)) + 1;
      pairs[(size_t)r * per + k] = make_int2(std::min(a, c), std::max(a, c));
    }
  if (nblk == 1) {  // cannot happen: nblk is even and >= 2
    return fail(ctx, MS_ERR_ARG, "jacobi: no blocks");
  }
  void* wsp = nullptr;
  void* wsc = nullptr;
  const size_t pbytes = pairs.size() * sizeof(int2);
  const bool have = ctx->ws.size() > 10 && ctx->ws[10] && ctx->jacobi_n == n;
  MS_TRY(workspace(ctx, 10, pbytes, &wsp));
  MS_TRY(workspace(ctx, 11, (size_t)nb * (max_sweeps + nblk + (size_t)rounds * per) * sizeof(int32_t), &wsc));
  if (!have || wsp != ctx->jacobi_pairs) {   // the schedule depends on n only: upload once
    MS_TRY(upload(ctx, wsp, pairs.data(), pbytes));
    ctx->jacobi_n = n;
    ctx->jacobi_pairs = wsp;
  }
  // [counters: nb x max_sweeps][block stamps: nb x nblk][pair stamps: nb x rounds x per]
  int32_t* cnt0 = static_cast<int32_t*>(wsc);
  const int64_t nrec = (int64_t)nb * (nblk + (int64_t)rounds * per);
  MS_TRY(launch_fill_i32(ctx, (int64_t)nb * max_sweeps, cnt0, 0));
  MS_TRY(launch_fill_i32(ctx, nrec, cnt0 + (int64_t)nb * max_sweeps, -1));
  JacobiArgs a;
  a.W = W;
  a.n = n;
  a.nb_real = nb_real;
  a.counter = cnt0;
  a.max_sweeps = max_sweeps;
  a.tol = std::max(1e-14, 4.0 * 2.220446049250313e-16 * std::sqrt((double)n));
  a.bmod = cnt0 + (int64_t)nb * max_sweeps;
  a.pconv = a.bmod + (int64_t)nb * nblk;
  a.nblk = nblk;
  a.npairs = rounds * per;
  a.per = per;
  for (int s = 0; s < max_sweeps; ++s) {
    a.sweep = s;
    for (int r = 0; r < rounds; ++r) {
      a.round = r;
      a.pairs = static_cast<const int2*>(wsp) + (size_t)r * per;
      Prof prof(ctx, PC_JACOBI, 2.0 * 8.0 * PW * PW * (double)n * per * nb, 3.0 * 16.0 * PW * (double)n * per * nb);
      hipLaunchKernelGGL(k_jacobi_round, dim3(per, nb), dim3(256), 0, ctx->stream, a);
      MS_TRY(check_launch(ctx, "jacobi round"));
    }
  }
  hipLaunchKernelGGL(k_jacobi_normalize, dim3((n + 255) / 256, nb), dim3(256), 0, ctx->stream, W, n, a.counter,
                     max_sweeps, status);
  MS_TRY(check_launch(ctx, "jacobi normalize"));
  // Z = H U (unsorted), then Rayleigh quotients
  GemmArgs g;
  g.M = n; g.N = n; g.K = n;
  g.A = H; g.lda = n; g.sA = (int64_t)n * n;
  g.B = W; g.ldb = n; g.sB = (int64_t)n * n;
  g.C = Z; g.ldc = n; g.sC = (int64_t)n * n;
  g.batch = nb;
  g.prof = PC_PREP_GEMM;
  MS_TRY(zgemm(ctx, g));
  const size_t shmem = (size_t)n * (sizeof(double) + sizeof(int));
  if (shmem > 64 * 1024) return fail(ctx, MS_ERR_UNSUPPORTED, "eigensolver size %d too large", n);
  hipLaunchKernelGGL(k_jacobi_emit, dim3(nb), dim3(256), shmem, ctx->stream, W, Z, n, eps_out, eps_stride, U,
                     u_stride);
  return check_launch(ctx, "jacobi emit");
}

ms_status launch_minmax(ms_ctx ctx, int64_t count, const int32_t* v, int32_t* out2) {
  hipLaunchKernelGGL(k_minmax, dim3(1), dim3(256), 0, ctx->stream, count, v, out2);
  return check_launch(ctx, "minmax");
}

ms_status launch_copy_boundary_overlaps(ms_ctx ctx, int n, const double2* U, double2* O, int conj_transpose) {
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(k_copy_overlap, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, ctx->stream, n, U, O,
                     conj_transpose);
  return check_launch(ctx, "boundary overlap");
}

}  // namespace ms
