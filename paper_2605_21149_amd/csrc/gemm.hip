// FP64 GEMM on the CDNA4 matrix cores: C = alpha * op(A) op(B) + beta * C.
//
// Workgroup tile BM x BN, 4 waves in a 2 x 2 arrangement, each wave owning a (BM/2) x (BN/2)
// sub-tile built from 16 x 16 blocks of v_mfma_f64_16x16x4.  K advances in slabs of 16 staged
// through LDS (double-buffered: the next slab is fetched into registers while the current one
// feeds the MFMAs).  Operands may be stored either way round (at/bt), so the same kernel serves
// the Cholesky trailing update (A B^T), the triangular-solve updates (A B) and Z = G^T G (A^T B).
//
// FP64 MFMA lane layout (measured on gfx950): lane l supplies A[l%16][l/16] and B[l/16][l%16];
// output register r of lane l is D[l/16 + 4r][l%16].
#include "cf_internal.h"

namespace cf {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

struct GemmArgs {
  int64_t M, N, K;
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  double* C; int64_t ldc;
  double alpha, beta;
  int lower;
  int64_t sA, sB, sC;
  int tiles_n;
};

template <int BM, int BN, bool AT, bool BT>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  constexpr int BK = 16, PAD = 1;
  constexpr int WM = BM / 2, WN = BN / 2, MI = WM / 16, NI = WN / 16;
  constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
  __shared__ double As[2][BK][BM + PAD];
  __shared__ double Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int tile_m = blockIdx.x / g.tiles_n, tile_n = blockIdx.x % g.tiles_n;
  const int64_t i0 = (int64_t)tile_m * BM, j0 = (int64_t)tile_n * BN;
  if (g.lower && j0 >= i0 + BM) return;            // tile strictly above the diagonal
  const int64_t z = blockIdx.z;
  const double* __restrict__ A = g.A + z * g.sA;
  const double* __restrict__ B = g.B + z * g.sB;
  double* __restrict__ C = g.C + z * g.sC;
  const int64_t M = g.M, N = g.N, K = g.K;

  double ra[LA], rb[LB];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < LA; ++p) {
      int idx = p * 256 + tid;
      int ii = AT ? (idx % BM) : (idx / BK);
      int kk = AT ? (idx / BM) : (idx % BK);
      int64_t gi = i0 + ii, gk = k0 + kk;
      ra[p] = (gi < M && gk < K) ? (AT ? A[gk * g.lda + gi] : A[gi * g.lda + gk]) : 0.0;
    }
#pragma unroll
    for (int p = 0; p < LB; ++p) {
      int idx = p * 256 + tid;
      int jj = BT ? (idx / BK) : (idx % BN);
      int kk = BT ? (idx % BK) : (idx / BN);
      int64_t gj = j0 + jj, gk = k0 + kk;
      rb[p] = (gj < N && gk < K) ? (BT ? B[gj * g.ldb + gk] : B[gk * g.ldb + gj]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < LA; ++p) {
      int idx = p * 256 + tid;
      int ii = AT ? (idx % BM) : (idx / BK);
      int kk = AT ? (idx / BM) : (idx % BK);
      As[buf][kk][ii] = ra[p];
    }
#pragma unroll
    for (int p = 0; p < LB; ++p) {
      int idx = p * 256 + tid;
      int jj = BT ? (idx / BK) : (idx % BN);
      int kk = BT ? (idx % BK) : (idx / BN);
      Bs[buf][kk][jj] = rb[p];
    }
  };

  dbl4 acc[MI][NI];
#pragma unroll
  for (int a = 0; a < MI; ++a)
#pragma unroll
    for (int b = 0; b < NI; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

  const int64_t nk = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int64_t t = 0; t < nk; ++t) {
    const int cur = (int)(t & 1);
    if (t + 1 < nk) load((t + 1) * BK);
#pragma unroll
    for (int kq = 0; kq < BK / 4; ++kq) {
      const int kr = kq * 4 + (lane >> 4);
      double av[MI], bv[NI];
#pragma unroll
      for (int a = 0; a < MI; ++a) av[a] = As[cur][kr][wr * WM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < NI; ++b) bv[b] = Bs[cur][kr][wc * WN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < MI; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (t + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  const double alpha = g.alpha, beta = g.beta;
#pragma unroll
  for (int a = 0; a < MI; ++a) {
#pragma unroll
    for (int b = 0; b < NI; ++b) {
      const int64_t col = j0 + wc * WN + b * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = i0 + wr * WM + a * 16 + (lane >> 4) + 4 * r;
        if (row < M && col < N) {
          double v = alpha * acc[a][b][r];
          double* p = C + row * g.ldc + col;
          if (beta != 0.0) v = fma(beta, *p, v);
          *p = v;
        }
      }
    }
  }
}

template <int BM, int BN>
hipError_t launch_tile(const GemmDesc& d, hipStream_t s) {
  GemmArgs g;
  g.M = d.M; g.N = d.N; g.K = d.K;
  g.A = d.A; g.lda = d.lda; g.B = d.B; g.ldb = d.ldb; g.C = d.C; g.ldc = d.ldc;
  g.alpha = d.alpha; g.beta = d.beta; g.lower = d.lower;
  g.sA = d.sA; g.sB = d.sB; g.sC = d.sC;
  const int64_t tm = (d.M + BM - 1) / BM, tn = (d.N + BN - 1) / BN;
  g.tiles_n = (int)tn;
  dim3 grid((unsigned)(tm * tn), 1, d.batch > 0 ? d.batch : 1), block(256);
  if (d.at && d.bt) hipLaunchKernelGGL((k_gemm<BM, BN, true, true>), grid, block, 0, s, g);
  else if (d.at) hipLaunchKernelGGL((k_gemm<BM, BN, true, false>), grid, block, 0, s, g);
  else if (d.bt) hipLaunchKernelGGL((k_gemm<BM, BN, false, true>), grid, block, 0, s, g);
  else hipLaunchKernelGGL((k_gemm<BM, BN, false, false>), grid, block, 0, s, g);
  return hipGetLastError();
}

}  // namespace

hipError_t gemm_f64(const GemmDesc& d, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  if (d.K <= 0) {
    // C = beta * C (alpha term vanishes): not needed by any caller; treat as a no-op only when beta == 1
    return d.beta == 1.0 ? hipSuccess : hipErrorInvalidValue;
  }
  const int64_t batch = d.batch > 0 ? d.batch : 1;
  const int64_t big = ((d.M + 127) / 128) * ((d.N + 127) / 128) * batch;
  if (big >= 480) return launch_tile<128, 128>(d, s);
  return launch_tile<64, 64>(d, s);
}

}  // namespace cf
