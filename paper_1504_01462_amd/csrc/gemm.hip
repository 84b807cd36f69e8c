// Batched complex GEMM on CDNA4 matrix cores.
//
// C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b], row-major, op in {N, T, C}.
// Complex operands are split into real/imaginary planes when staged into LDS;
// each 16x16x4 complex block is three real MFMAs (Gauss's product)
//   P1 += Ar Br,   P2 += Ai Bi,   P3 += (Ar + Ai)(Br + Bi);   Cr = P1 - P2,   Ci = P3 - P1 - P2
// (v_mfma_f64_16x16x4f64 for complex128, v_mfma_f32_16x16x4f32 for complex64:
// FP32 accumulation inside each K-slab of 16, each product's slabs summed in FP64).  Three
// products instead of four take a quarter of the matrix-core work; the imaginary part's
// rounding error is bounded by eps sum (|Ar| + |Ai|)(|Br| + |Bi|) instead of
// eps sum (|Ar| |Bi| + |Ai| |Br|).  Operand layouts of both: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; the accumulator layouts differ
// (see Mfma<T>::crow).  Each wave owns a 32 x 32 sub-tile: 64 x 64 tiles with 4 waves in a
// 2 x 2 grid, or (FP64) 128 x 64 tiles with 8 waves in a 4 x 2 grid.  Global->LDS staging is
// register double-buffered (the next K-slab is fetched while the current one is used).
//
// The fold's interface product (ROLE 1) generates its B operand while staging it:
//   B_b[m][j] = O[j][m] (kp_b[j] - kq_b[m])          j <  nh   (C-)
//   B_b[m][j] = O[j'][m] (kp_b[j'] + kq_b[m]), 0 at m = j'   j = nh + j'  (C+ off its diagonal)
// from the shared FP64 overlap O and each batch entry's wavevectors, computed in FP64 and
// rounded to the MFMA type when stored into LDS.  A tile's columns are BN/2 columns of C-
// and the same BN/2 columns of C+, so each O element is loaded once and staged twice.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include <hip/hip_ext.h>

#include "ms_internal.h"

namespace ms {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4_t acc_t;
  typedef double2 c_t;
  static __device__ __forceinline__ d4_t mac(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator element v of `lane` holds row (lane / 16) + 4 v, column lane % 16
  static __device__ __forceinline__ int crow(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef f4_t acc_t;
  typedef float2 c_t;
  static __device__ __forceinline__ f4_t mac(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element v of `lane` holds row 4 (lane / 16) + v, column lane % 16
  static __device__ __forceinline__ int crow(int lane, int v) { return 4 * (lane >> 4) + v; }
};

struct KParams {
  int M, N, K, opA, opB;
  const void* A;
  int64_t lda, sA;
  const void* B;
  int64_t ldb, sB;
  double2* C;
  int64_t ldc, sC;
  double2 alpha, beta;
  // generated B (ROLE 1): wavevectors of batch entry b at kp + b sk, kq + b sk; N = 2 nh
  const double2* kp;
  const double2* kq;
  int64_t sk;
  int nh;
  // fused fold epilogue (generated B only; ey null: plain W)
  const double2* ey;
  int64_t eldy, esy;
  const double2* epq;
  const int32_t* esel;
  int ecap;
};

// complex product with its two fused multiply-adds written out, so every instantiation of the
// kernel rounds it the same way (the compiler is otherwise free to contract either product)
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {   // fused multiply-adds written out
  const double d = fma(b.x, b.x, b.y * b.y);
  return make_double2(fma(a.x, b.x, a.y * b.y) / d, fma(a.y, b.x, -(a.x * b.y)) / d);
}

constexpr int BK = 16;

// Tile BM x BN, WM x WN waves (each owning a (BM/WM) x (BN/WN) sub-tile).
// LDS rows are padded by one element so the transposing stores of the
// staging pass spread over the banks.  Blocks are launched as a 1D grid whose
// index is remapped so that consecutive logical tiles (same A row-panel, all
// column tiles) land on the same XCD and share its L2.  ROLE 1 is the fold's
// interface product with its generated B operand; otherwise ROLE does not change
// the code: it gives the LU's trailing updates (2) their own kernel names in
// kernel traces.
template <typename T, int BM, int BN, int WM, int WN, int ROLE>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm(KParams p, int ntn, int ntm, int total) {
  typedef typename Mfma<T>::c_t CT;
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 16, FN = TN / 16;
  constexpr int EA = BM * BK / NT, EB = BN * BK / NT;
  constexpr int PA = BM + 1, PB = BN + 1;
  __shared__ T As[2][2][BK][PA];   // [stage][re/im][k][m]
  __shared__ T Bs[2][2][BK][PB];

  // XCD-aware remap of the linear block index
  const int hw = blockIdx.x;
  int lid = hw;
  if ((total & 7) == 0) lid = (hw & 7) * (total >> 3) + (hw >> 3);
  int tn, tm;
  int64_t b;
  if constexpr (ROLE == 1) {
    // interface product: row tiles r = (batch entry, tm) of all entries share the O panels, so
    // runs of GROUP consecutive row tiles take each column tile in turn (GROUP blocks on one
    // XCD read the same O panel while their A panels stay in its L2)
    constexpr int GROUP = 8;
    const int nrow = total / ntn;
    const int per = GROUP * ntn;
    const int first = (lid / per) * GROUP;
    const int gsz = min(nrow - first, GROUP);
    const int r = first + (lid % per) % gsz;
    tn = (lid % per) / gsz;
    tm = r % ntm;
    b = r / ntm;
  } else {
    tn = lid % ntn;
    tm = (lid / ntn) % ntm;
    b = lid / (ntn * ntm);
  }

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / WN) * TM, wn0 = (wave % WN) * TN;
  const int m0 = tm * BM, n0 = tn * BN;
  constexpr bool GEN = ROLE == 1;   // generated B (opB = T semantics, FP64 source)
  const CT* A = static_cast<const CT*>(p.A) + b * p.sA;
  const CT* B = static_cast<const CT*>(p.B) + b * p.sB;
  const double2* Bd = static_cast<const double2*>(p.B);   // generated B: the shared overlap O
  double2* C = p.C + b * p.sC;
  const bool use_beta = (p.beta.x != 0.0 || p.beta.y != 0.0);
  // FP64: alpha is applied to A as it is staged and beta C is loaded into the
  // accumulators before the K loop, so the C read overlaps the first K-slabs
  // instead of trailing the last one.  FP32 accumulators keep the epilogue form.
  constexpr bool kFold = std::is_same<T, double>::value;
  const bool scale_a = !(p.alpha.x == 1.0 && p.alpha.y == 0.0);

  // Register double buffer.  load() issues the global loads of a K-slab with
  // indices clamped into the matrices (every address valid, no branch), so the
  // loads stay in flight while the MFMAs of the current slab run; stash()
  // consumes them afterwards: zeroes the out-of-range elements, conjugates,
  // scales by alpha and stores the split planes into LDS.
  CT ra[EA], rb[EB];
  // generated B: each thread's B elements keep their column j across K-slabs and share one
  // K offset (NT is a multiple of BK), so kp is loaded once and kq once per slab
  // (generated B: tile column c < BN/2 is C- column n0h + c, c >= BN/2 is C+ column
  // n0h + c - BN/2, with n0h = tn BN/2; a thread loads EB/2 O elements per slab)
  constexpr int BNH = BN / 2, EBH = EB / 2;
  const int n0h = tn * BNH;
  double2 rbd[GEN ? EBH : 1], kpv[GEN ? EBH : 1], rkq = make_double2(0.0, 0.0);
  const double2* kpb = GEN ? p.kp + b * p.sk : nullptr;
  const double2* kqb = GEN ? p.kq + b * p.sk : nullptr;
  if constexpr (GEN) {
#pragma unroll
    for (int e = 0; e < EBH; ++e) kpv[e] = kpb[min(n0h + (tid + NT * e) / BK, p.nh - 1)];
  }
  // generated B (op(A) = A): every thread's A and O elements keep their rows across K-slabs
  // and share one K offset (tid mod BK), so the row addresses are formed once, here
  const CT* arow[GEN ? EA : 1];
  const double2* brow[GEN ? EBH : 1];
  if constexpr (GEN) {
#pragma unroll
    for (int e = 0; e < EA; ++e) arow[e] = A + (int64_t)min(m0 + (tid + NT * e) / BK, p.M - 1) * p.lda;
#pragma unroll
    for (int e = 0; e < EBH; ++e) brow[e] = Bd + (int64_t)min(n0h + (tid + NT * e) / BK, p.nh - 1) * p.ldb;
  }
  auto load = [&](int k0) {
    if constexpr (GEN) {
      const int gk = min(k0 + tid % BK, p.K - 1);
#pragma unroll
      for (int e = 0; e < EA; ++e) ra[e] = arow[e][gk];
      rkq = kqb[gk];
#pragma unroll
      for (int e = 0; e < EBH; ++e) rbd[e] = brow[e][gk];
      return;
    }
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + NT * e;
      int i, k;
      if (p.opA == OP_N) { i = idx / BK; k = idx % BK; } else { k = idx / BM; i = idx % BM; }
      const int gi = min(m0 + i, p.M - 1), gk = min(k0 + k, p.K - 1);
      ra[e] = (p.opA == OP_N) ? A[(int64_t)gi * p.lda + gk] : A[(int64_t)gk * p.lda + gi];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + NT * e;
      int j, k;
      if (p.opB == OP_N) { k = idx / BN; j = idx % BN; } else { j = idx / BK; k = idx % BK; }
      const int gj = min(n0 + j, p.N - 1), gk = min(k0 + k, p.K - 1);
      rb[e] = (p.opB == OP_N) ? B[(int64_t)gk * p.ldb + gj] : B[(int64_t)gj * p.ldb + gk];
    }
  };
  auto stash = [&](int st, int k0) {
    const bool aN = GEN || p.opA == OP_N;
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + NT * e;
      int i, k;
      if (aN) { i = idx / BK; k = idx % BK; } else { k = idx / BM; i = idx % BM; }
      const bool ok = m0 + i < p.M && k0 + k < p.K;
      T re = ok ? ra[e].x : (T)0, im = ok ? ra[e].y : (T)0;
      if (!GEN && p.opA == OP_C) im = -im;
      if (kFold && scale_a) {   // alpha op(A), staged (fused multiply-adds written out)
        const T r2 = fma((T)p.alpha.x, re, -((T)p.alpha.y * im));
        im = fma((T)p.alpha.x, im, (T)p.alpha.y * re);
        re = r2;
      }
      As[st][0][k][i] = re;
      As[st][1][k][i] = im;
    }
    if constexpr (GEN) {
#pragma unroll
      for (int e = 0; e < EBH; ++e) {
        const int idx = tid + NT * e;
        const int j = idx / BK, k = idx % BK;
        const int gj = n0h + j, gk = k0 + k;
        const double2 vm = zmul(rbd[e], make_double2(kpv[e].x - rkq.x, kpv[e].y - rkq.y));
        const double2 vp = zmul(rbd[e], make_double2(kpv[e].x + rkq.x, kpv[e].y + rkq.y));
        const bool ok = gj < p.nh && gk < p.K;
        const bool okp = ok && gk != gj;   // C+ without its diagonal
        Bs[st][0][k][j] = ok ? (T)vm.x : (T)0;
        Bs[st][1][k][j] = ok ? (T)vm.y : (T)0;
        Bs[st][0][k][BNH + j] = okp ? (T)vp.x : (T)0;
        Bs[st][1][k][BNH + j] = okp ? (T)vp.y : (T)0;
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + NT * e;
      int j, k;
      if (p.opB == OP_N) { k = idx / BN; j = idx % BN; } else { j = idx / BK; k = idx % BK; }
      const bool ok = n0 + j < p.N && k0 + k < p.K;
      T re = ok ? rb[e].x : (T)0, im = ok ? rb[e].y : (T)0;
      if (p.opB == OP_C) im = -im;
      Bs[st][0][k][j] = re;
      Bs[st][1][k][j] = im;
    }
  };

  // Gauss's three-product form: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi);
  // Re = P1 - P2, Im = P3 - P1 - P2
  acc_t cr[FM][FN], ci[FM][FN], c3[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int c = 0; c < FN; ++c) {
      cr[a][c] = acc_t{0, 0, 0, 0};
      ci[a][c] = acc_t{0, 0, 0, 0};
      c3[a][c] = acc_t{0, 0, 0, 0};
    }
  // FP32 MFMA: each K-slab accumulates in FP32 (four MFMA steps), and the slabs of each of the
  // three products are summed in FP64 (sr, si, s3: P1, P2, P3), so the FP32 rounding chain of
  // an element is 4 long instead of K / 4; the products are combined once, after the K loop
  // (three sums take two FP64 operations per element and slab fewer than two combined ones)
  constexpr bool kSlab64 = !kFold;
  double sr[kSlab64 ? FM : 1][kSlab64 ? FN : 1][4], si[kSlab64 ? FM : 1][kSlab64 ? FN : 1][4],
      s3[kSlab64 ? FM : 1][kSlab64 ? FN : 1][4];
  if constexpr (kSlab64) {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int c = 0; c < FN; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) sr[a][c][v] = si[a][c][v] = s3[a][c][v] = 0.0;
  }

  // two LDS stages: compute on stage `cur` while the next K-slab is stored into the
  // other one; one barrier per slab
  if (p.K > 0) load(0);
  if (kFold && use_beta) {   // C loads unconditional (clamped) so they are all in flight at once
    const bool beta_one = p.beta.x == 1.0 && p.beta.y == 0.0;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int c = 0; c < FN; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = m0 + wm0 + a * 16 + Mfma<T>::crow(lane, v);
          const int col = n0 + wn0 + c * 16 + (lane & 15);
          const double2 o = C[(int64_t)min(row, p.M - 1) * p.ldc + min(col, p.N - 1)];
          const bool ok = row < p.M && col < p.N;
          const double re = beta_one ? o.x : fma(p.beta.x, o.x, -(p.beta.y * o.y));
          const double im = beta_one ? o.y : fma(p.beta.x, o.y, p.beta.y * o.x);
          cr[a][c][v] = ok ? re : 0.0;
          ci[a][c][v] = 0.0;
          c3[a][c][v] = ok ? re + im : 0.0;
        }
  }
  stash(0, 0);
  if (BK < p.K) load(BK);
  __syncthreads();
  int cur = 0;
  for (int k0 = 0; k0 < p.K; k0 += BK) {
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      T ar[FM], ai[FM], as[FM], br[FN], bi[FN], bs[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        ar[a] = As[cur][0][kr][wm0 + a * 16 + (lane & 15)];
        ai[a] = As[cur][1][kr][wm0 + a * 16 + (lane & 15)];
        as[a] = ar[a] + ai[a];
      }
#pragma unroll
      for (int c = 0; c < FN; ++c) {
        br[c] = Bs[cur][0][kr][wn0 + c * 16 + (lane & 15)];
        bi[c] = Bs[cur][1][kr][wn0 + c * 16 + (lane & 15)];
        bs[c] = br[c] + bi[c];
      }
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int c = 0; c < FN; ++c) {
          cr[a][c] = Mfma<T>::mac(ar[a], br[c], cr[a][c]);
          ci[a][c] = Mfma<T>::mac(ai[a], bi[c], ci[a][c]);
          c3[a][c] = Mfma<T>::mac(as[a], bs[c], c3[a][c]);
        }
    }
    if constexpr (kSlab64) {
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int c = 0; c < FN; ++c) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double p1 = (double)cr[a][c][v], p2 = (double)ci[a][c][v], p3 = (double)c3[a][c][v];
            sr[a][c][v] += p1;
            si[a][c][v] += p2;
            s3[a][c][v] += p3;
          }
          cr[a][c] = acc_t{0, 0, 0, 0};
          ci[a][c] = acc_t{0, 0, 0, 0};
          c3[a][c] = acc_t{0, 0, 0, 0};
        }
    }
    if (k0 + BK < p.K) {
      stash(cur ^ 1, k0 + BK);              // slab k0+BK (already in registers)
      if (k0 + 2 * BK < p.K) load(k0 + 2 * BK);
    }
    __syncthreads();
    cur ^= 1;
  }

#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int c = 0; c < FN; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm0 + a * 16 + Mfma<T>::crow(lane, v);
        int col = n0 + wn0 + c * 16 + (lane & 15);
        bool col_ok = col < p.N;
        if constexpr (GEN) {   // tile column -> C- or C+ column
          const int lc = wn0 + c * 16 + (lane & 15);
          const int h = lc >= BNH ? lc - BNH : lc;
          col_ok = n0h + h < p.nh;
          col = (lc >= BNH ? p.nh : 0) + n0h + h;
        }
        if (row < p.M && col_ok) {
          if constexpr (GEN) {
            if (p.ey) {   // the fold's augmented-matrix columns (see GemmArgs)
              double wr, wi;
              if constexpr (kSlab64) {
                wr = sr[a][c][v] - si[a][c][v];
                wi = s3[a][c][v] - sr[a][c][v] - si[a][c][v];
              } else {
                const double p1 = (double)cr[a][c][v], p2 = (double)ci[a][c][v], p3 = (double)c3[a][c][v];
                wr = p1 - p2;
                wi = p3 - p1 - p2;
              }
              const int lc = wn0 + c * 16 + (lane & 15);
              const bool plus = lc >= BNH;       // W+ column (Phi_B^T), else W- (Phi_A^T)
              const int j = n0h + (plus ? lc - BNH : lc), i = row;
              const double2 kpj = kpb[j], kqi = kqb[i];
              const double2 ot = Bd[(int64_t)j * p.ldb + i];
              const double2* Yb = p.ey + b * p.esy + (int64_t)i * p.eldy;
              const double2* Pb = p.epq + b * p.sk;
              const double2 pk = zmul(Pb[i], kqi);
              double2 out = make_double2(wr, wi);
              if (!plus) {
                out = zadd(out, zmul(ot, zadd(kpj, kqi)));
              } else {
                out = zadd(out, zmul(ot, zsub(kpj, kqi)));
                const double2 rho = zdiv(zmul(zmul(pk, Yb[j]), Pb[j]), kqb[j]);
                out = zadd(out, zmul(rho, zmul(Bd[(int64_t)j * p.ldb + j], zadd(kpj, kqb[j]))));
              }
              if (p.esel) {
                const int32_t* se = p.esel + b * (int64_t)(p.ecap + 1);
                const int nsel = se[0];
                for (int q = 0; q < nsel; ++q) {
                  const int m = se[1 + q];
                  if (plus && m == j) continue;
                  const double2 rm = zdiv(zmul(zmul(pk, Yb[m]), Pb[m]), kqb[m]);
                  const double2 ojm = Bd[(int64_t)j * p.ldb + m];
                  out = zadd(out, zmul(rm, zmul(ojm, plus ? zadd(kpj, kqb[m]) : zsub(kpj, kqb[m]))));
                }
              }
              C[(int64_t)row * p.ldc + col] = out;
              continue;
            }
          }
          if (kFold) {
            const double p1 = (double)cr[a][c][v], p2 = (double)ci[a][c][v], p3 = (double)c3[a][c][v];
            C[(int64_t)row * p.ldc + col] = make_double2(p1 - p2, p3 - p1 - p2);
            continue;
          }
          double re, im;
          if constexpr (kSlab64) {
            re = sr[a][c][v] - si[a][c][v];
            im = s3[a][c][v] - sr[a][c][v] - si[a][c][v];
          } else {
            const double p1 = (double)cr[a][c][v], p2 = (double)ci[a][c][v], p3 = (double)c3[a][c][v];
            re = p1 - p2;
            im = p3 - p1 - p2;
          }
          double2 out;
          out.x = p.alpha.x * re - p.alpha.y * im;
          out.y = p.alpha.x * im + p.alpha.y * re;
          double2* dst = C + (int64_t)row * p.ldc + col;
          if (use_beta) {
            const double2 o = *dst;
            out.x += p.beta.x * o.x - p.beta.y * o.y;
            out.y += p.beta.x * o.y + p.beta.y * o.x;
          }
          *dst = out;
        }
      }
}

template <typename T, int BM, int BN, int WM, int WN, int ROLE>
ms_status launch(ms_ctx ctx, const KParams& p, int batch, const Prof& prof) {
  // generated B: a tile covers BN/2 columns of each half
  const int ntn = ROLE == 1 ? (p.nh + BN / 2 - 1) / (BN / 2) : (p.N + BN - 1) / BN, ntm = (p.M + BM - 1) / BM;
  const int64_t total = (int64_t)ntn * ntm * batch;
  if (total > 0x7fffffff) return fail(ctx, MS_ERR_UNSUPPORTED, "gemm grid too large");
  if (prof.a)   // timed: the events bracket the kernel's execution
    hipExtLaunchKernelGGL((k_gemm<T, BM, BN, WM, WN, ROLE>), dim3((unsigned)total), dim3(64 * WM * WN), 0,
                          ctx->stream, prof.a, prof.b, 0, p, ntn, ntm, (int)total);
  else
    hipLaunchKernelGGL((k_gemm<T, BM, BN, WM, WN, ROLE>), dim3((unsigned)total), dim3(64 * WM * WN), 0, ctx->stream,
                       p, ntn, ntm, (int)total);
  return check_launch(ctx, "gemm");
}

template <typename T>
ms_status run(ms_ctx ctx, const GemmArgs& g) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return MS_OK;
  const bool gen = g.kp != nullptr;
  if (gen && (g.N % 2 != 0 || g.kq == nullptr || g.opB != OP_T || g.sB != 0 || g.beta.x != 0.0 || g.beta.y != 0.0 ||
              g.alpha.x != 1.0 || g.alpha.y != 0.0 || g.opA != OP_N))
    return fail(ctx, MS_ERR_ARG, "generated-B product: shared O^T, N = 2 nh, no alpha/beta");
  KParams p{g.M, g.N, std::max(g.K, 0), g.opA, g.opB, g.A, g.lda, g.sA, g.B, g.ldb, g.sB, g.C, g.ldc, g.sC, g.alpha,
            g.beta, g.kp, g.kq, g.sk, g.N / 2, gen ? g.ey : nullptr, g.eldy, g.esy, g.epq, g.esel, g.ecap};
  // algorithmic bytes: A and C per batch entry; a shared B (stride 0) once; the fused fold
  // epilogue also reads each entry's state Y (M x K)
  const double bytes_b = gen ? 16.0 * p.K * (g.N / 2) + 2.0 * 16.0 * g.batch * (p.K + g.N / 2) +
                                   (g.ey ? 16.0 * g.batch * (double)g.M * p.K : 0.0)
                             : (double)(g.sB == 0 ? 1 : g.batch) * sizeof(typename Mfma<T>::c_t) * p.K * g.N;
  Prof prof(ctx, g.prof, 8.0 * g.M * (double)g.N * p.K * g.batch,
            (double)g.batch * sizeof(typename Mfma<T>::c_t) * ((double)g.M * p.K) + bytes_b +
                (double)g.batch * 16.0 * g.M * g.N * ((g.beta.x != 0.0 || g.beta.y != 0.0) ? 2 : 1),
            true);
  // Tile edge: the tuned choice for the fold group's basis size (ms_autotune / ms_set_tiles),
  // else 64 x 64 (4 waves, two workgroups per CU), which timed faster than 128 x 64 (8 waves,
  // one workgroup per CU) for every role at N_G = 1200.  Every wave owns a 32 x 32 sub-tile in
  // both shapes and every element is accumulated in the same order, so the choice never
  // changes a result.
  static const int tile_env = [] {   // MS_GEMM_TILE=64: 64 x 64 tiles everywhere
    const char* e = getenv("MS_GEMM_TILE");
    return e ? atoi(e) : 0;
  }();
  int tile = 0;
  if (ctx->tile_n > 0)
    for (const auto& t : ctx->tiles)
      if (t.n == ctx->tile_n)
        tile = g.prof == PC_IFACE_GEMM ? t.iface
                                       : (g.prof == PC_LU_UPDATE ? t.lu_update : (g.prof == PC_LU_INNER ? t.lu_inner : 0));
  if (tile_env == 64) tile = 64;
  if (tile == 0) tile = 64;
  // FP32 MFMA keeps FP64 sums of its K-slabs (three per element): 64 x 64 tiles always
  if constexpr (!std::is_same<T, double>::value) {
    if (gen) return launch<T, 64, 64, 2, 2, 1>(ctx, p, g.batch, prof);
    return g.prof == PC_LU_UPDATE ? launch<T, 64, 64, 2, 2, 2>(ctx, p, g.batch, prof)
                                  : launch<T, 64, 64, 2, 2, 0>(ctx, p, g.batch, prof);
  } else {
    const bool big = tile == 128;   // 128 x 64, 8 waves
    if (g.prof == PC_LU_UPDATE)
      return big ? launch<T, 128, 64, 4, 2, 2>(ctx, p, g.batch, prof)
                 : launch<T, 64, 64, 2, 2, 2>(ctx, p, g.batch, prof);
    if (gen)
      return big ? launch<T, 128, 64, 4, 2, 1>(ctx, p, g.batch, prof)
                 : launch<T, 64, 64, 2, 2, 1>(ctx, p, g.batch, prof);
    return big ? launch<T, 128, 64, 4, 2, 0>(ctx, p, g.batch, prof) : launch<T, 64, 64, 2, 2, 0>(ctx, p, g.batch, prof);
  }
}

}  // namespace

ms_status zgemm(ms_ctx ctx, const GemmArgs& g) { return run<double>(ctx, g); }
ms_status cgemm32(ms_ctx ctx, const GemmArgs& g) { return run<float>(ctx, g); }

}  // namespace ms
