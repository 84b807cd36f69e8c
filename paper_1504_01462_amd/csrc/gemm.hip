// Batched complex GEMM on CDNA4 matrix cores.
//
// C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b], row-major, op in {N, T, C}.
// Complex operands are split into real/imaginary planes when staged into LDS;
// each 16x16x4 complex block is four real MFMAs
//   Cr += Ar Br - Ai Bi,   Ci += Ar Bi + Ai Br
// (v_mfma_f64_16x16x4f64 for complex128, v_mfma_f32_16x16x4f32 with FP32
// accumulation for complex64).  Operand layouts of both: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; the accumulator layouts differ
// (see Mfma<T>::crow).  Workgroup = 4 wave64s in a 2x2 grid; each wave
// owns a (BM/2) x (BN/2) sub-tile.  Global->LDS staging is register
// double-buffered (the next K-slab is fetched while the current one is used).
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
};

constexpr int BK = 16;
constexpr int NT = 256;

template <typename T, int BM, int BN>
__global__ __launch_bounds__(NT) void k_gemm(KParams p) {
  typedef typename Mfma<T>::c_t CT;
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int TM = BM / 2, TN = BN / 2;
  constexpr int FM = TM / 16, FN = TN / 16;
  constexpr int EA = BM * BK / NT, EB = BN * BK / NT;
  __shared__ T As[2][BK][BM];
  __shared__ T Bs[2][BK][BN];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * TM, wn0 = (wave & 1) * TN;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int64_t b = blockIdx.z;
  const CT* A = static_cast<const CT*>(p.A) + b * p.sA;
  const CT* B = static_cast<const CT*>(p.B) + b * p.sB;

  CT ra[EA], rb[EB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + NT * e;
      int i, k;
      if (p.opA == OP_N) { i = idx / BK; k = idx % BK; } else { k = idx / BM; i = idx % BM; }
      const int gi = m0 + i, gk = k0 + k;
      CT v;
      v.x = 0; v.y = 0;
      if (gi < p.M && gk < p.K) {
        v = (p.opA == OP_N) ? A[(int64_t)gi * p.lda + gk] : A[(int64_t)gk * p.lda + gi];
        if (p.opA == OP_C) v.y = -v.y;
      }
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + NT * e;
      int j, k;
      if (p.opB == OP_N) { k = idx / BN; j = idx % BN; } else { j = idx / BK; k = idx % BK; }
      const int gj = n0 + j, gk = k0 + k;
      CT v;
      v.x = 0; v.y = 0;
      if (gj < p.N && gk < p.K) {
        v = (p.opB == OP_N) ? B[(int64_t)gk * p.ldb + gj] : B[(int64_t)gj * p.ldb + gk];
        if (p.opB == OP_C) v.y = -v.y;
      }
      rb[e] = v;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + NT * e;
      int i, k;
      if (p.opA == OP_N) { i = idx / BK; k = idx % BK; } else { k = idx / BM; i = idx % BM; }
      As[0][k][i] = ra[e].x;
      As[1][k][i] = ra[e].y;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + NT * e;
      int j, k;
      if (p.opB == OP_N) { k = idx / BN; j = idx % BN; } else { j = idx / BK; k = idx % BK; }
      Bs[0][k][j] = rb[e].x;
      Bs[1][k][j] = rb[e].y;
    }
  };

  acc_t cr[FM][FN], ci[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int c = 0; c < FN; ++c) {
      cr[a][c] = acc_t{0, 0, 0, 0};
      ci[a][c] = acc_t{0, 0, 0, 0};
    }

  load(0);
  stash();
  __syncthreads();
  for (int k0 = 0; k0 < p.K; k0 += BK) {
    const bool more = k0 + BK < p.K;
    if (more) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      T ar[FM], ai[FM], nai[FM], br[FN], bi[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        ar[a] = As[0][kr][wm0 + a * 16 + (lane & 15)];
        ai[a] = As[1][kr][wm0 + a * 16 + (lane & 15)];
        nai[a] = -ai[a];
      }
#pragma unroll
      for (int c = 0; c < FN; ++c) {
        br[c] = Bs[0][kr][wn0 + c * 16 + (lane & 15)];
        bi[c] = Bs[1][kr][wn0 + c * 16 + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int c = 0; c < FN; ++c) {
          cr[a][c] = Mfma<T>::mac(ar[a], br[c], cr[a][c]);
          ci[a][c] = Mfma<T>::mac(ar[a], bi[c], ci[a][c]);
        }
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int c = 0; c < FN; ++c) {
          cr[a][c] = Mfma<T>::mac(nai[a], bi[c], cr[a][c]);
          ci[a][c] = Mfma<T>::mac(ai[a], br[c], ci[a][c]);
        }
    }
    __syncthreads();
    if (more) {
      stash();
      __syncthreads();
    }
  }

  double2* C = p.C + b * p.sC;
  const bool use_beta = (p.beta.x != 0.0 || p.beta.y != 0.0);
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int c = 0; c < FN; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm0 + a * 16 + Mfma<T>::crow(lane, v);
        const int col = n0 + wn0 + c * 16 + (lane & 15);
        if (row < p.M && col < p.N) {
          const double re = (double)cr[a][c][v], im = (double)ci[a][c][v];
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

template <typename T>
ms_status run(ms_ctx ctx, const GemmArgs& g) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return MS_OK;
  if (g.batch > 65535) return fail(ctx, MS_ERR_UNSUPPORTED, "gemm batch %d > 65535", g.batch);
  KParams p{g.M, g.N, g.K, g.opA, g.opB, g.A, g.lda, g.sA, g.B, g.ldb, g.sB, g.C, g.ldc, g.sC, g.alpha, g.beta};
  if (g.K <= 0) {  // C = beta C
    p.K = 0;
  }
  constexpr int BM = 64, BN = 64;
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, g.batch);
  Prof prof(ctx, g.prof, 8.0 * g.M * (double)g.N * g.K * g.batch,
            (double)g.batch * sizeof(typename Mfma<T>::c_t) * ((double)g.M * g.K + (double)g.K * g.N) +
                (double)g.batch * 16.0 * g.M * g.N * ((g.beta.x != 0.0 || g.beta.y != 0.0) ? 2 : 1));
  hipLaunchKernelGGL((k_gemm<T, BM, BN>), grid, dim3(NT), 0, ctx->stream, p);
  return check_launch(ctx, "gemm");
}

}  // namespace

ms_status zgemm(ms_ctx ctx, const GemmArgs& g) { return run<double>(ctx, g); }
ms_status cgemm32(ms_ctx ctx, const GemmArgs& g) { return run<float>(ctx, g); }

}  // namespace ms
