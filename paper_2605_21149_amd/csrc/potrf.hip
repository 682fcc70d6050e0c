// Blocked Cholesky C = L L^T, ln|C| from its diagonal, and forward substitution L^-1 Y.
//
// Right-looking, two-level blocking: 256-column outer panels whose 64-column diagonal blocks are
// factorised in LDS by one workgroup; the column panel below each block is solved row-parallel
// (X L11^-T, one row per lane, the row held in registers); the remaining columns of the outer
// panel and then the whole trailing matrix are updated with the FP64 matrix-core GEMM.
// The forward substitution L^-1 Y recurses on halves of the row range: leaves solve a 64-row
// block column-parallel (one right-hand side per lane), interior nodes are GEMM updates.
#include "cf_internal.h"
#include <climits>

namespace cf {
namespace {

constexpr int NB = kNB;          // 64
constexpr int OUTER = 256;       // outer panel width

// Factor the b x b (b <= 64) diagonal block at (c, c).  One barrier per column: the trailing
// update uses the unscaled column, a_rq -= a_rj a_qj / a_jj, and the scaled factor is written
// once at the end.
__global__ __launch_bounds__(256) void k_potrf_diag(double* A_base, int64_t lda, int64_t sA, int64_t c,
                                                    int b, double* dinv_base, int64_t sD,
                                                    double* ldpart_base, int64_t sL, int blk,
                                                    int* fail) {
  __shared__ double a[NB][NB + 1];
  const int tid = threadIdx.x;
  double* A = A_base + blockIdx.z * sA + c * lda + c;
  for (int idx = tid; idx < b * b; idx += 256) {
    int r = idx / b, q = idx % b;
    if (q <= r) a[r][q] = A[r * lda + q];
  }
  __syncthreads();
  for (int j = 0; j < b; ++j) {
    const double d = a[j][j];
    const int m = b - j - 1;
    if (m > 0) {
      const double inv = 1.0 / d;
      for (int idx = tid; idx < m * m; idx += 256) {
        int r = j + 1 + idx / m, q = j + 1 + idx % m;
        if (q <= r) a[r][q] -= a[r][j] * a[q][j] * inv;
      }
    }
    __syncthreads();
  }
  double* dinv = dinv_base + blockIdx.z * sD + c;
  for (int idx = tid; idx < b * b; idx += 256) {
    int r = idx / b, q = idx % b;
    if (q <= r) {
      double s = sqrt(a[q][q]);
      A[r * lda + q] = a[r][q] / s;
      if (r == q) dinv[q] = 1.0 / s;
    }
  }
  if (tid == 0) {
    double acc = 0.0;
    int bad = INT_MAX;
    for (int j = 0; j < b; ++j) {
      double d = a[j][j];
      if (!(d > 0.0) || !isfinite(d)) { if (bad == INT_MAX) bad = (int)c + j; }
      acc += 0.5 * log(d);
    }
    ldpart_base[blockIdx.z * sL + blk] = acc;
    if (bad != INT_MAX) atomicMin(fail, bad);
  }
}

// X (M x b rows below the diagonal block) <- X L11^-T.  64 rows per workgroup, one per lane.
__global__ __launch_bounds__(64) void k_trsm_rows(double* A_base, int64_t lda, int64_t sA, int64_t c,
                                                  int b, int64_t M, const double* dinv_base,
                                                  int64_t sD) {
  __shared__ double Ls[NB][NB + 1];
  __shared__ double Xs[NB][NB + 1];
  __shared__ double di[NB];
  const int t = threadIdx.x;
  double* A = A_base + blockIdx.z * sA;
  const double* L11 = A + c * lda + c;
  const double* dinv = dinv_base + blockIdx.z * sD + c;
  const int64_t r0 = c + b + (int64_t)blockIdx.x * NB;       // first row of this tile
  for (int r = 0; r < NB; ++r) {
    Ls[r][t] = (r < b && t < b) ? (t <= r ? L11[r * lda + t] : 0.0) : (r == t ? 1.0 : 0.0);
    int64_t gr = r0 + r;
    Xs[r][t] = (gr < c + b + M && t < b) ? A[gr * lda + c + t] : 0.0;
  }
  di[t] = t < b ? dinv[t] : 1.0;
  __syncthreads();
  double x[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) x[q] = Xs[t][q];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const double xj = x[j] * di[j];
    x[j] = xj;
#pragma unroll
    for (int i = j + 1; i < NB; ++i) x[i] = fma(-Ls[i][j], xj, x[i]);
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) Xs[t][q] = x[q];
  __syncthreads();
  for (int r = 0; r < NB; ++r) {
    int64_t gr = r0 + r;
    if (gr < c + b + M && t < b) A[gr * lda + c + t] = Xs[r][t];
  }
}

// G[r0:r0+b, :] <- L11^-1 Y[r0:r0+b, :], one right-hand side (column) per lane; the 64 x 64
// tile of Y is staged through LDS so that global loads and stores stay coalesced.
__global__ __launch_bounds__(64) void k_trsm_cols(const double* L_base, int64_t ldl, int64_t sL,
                                                  const double* dinv_base, int64_t sD, int64_t r0,
                                                  int b, const double* Y_base, int64_t ldy, int64_t sY,
                                                  double* G_base, int64_t ldg, int64_t sG,
                                                  int64_t ncol) {
  __shared__ double Ls[NB][NB + 1];
  __shared__ double Xs[NB][NB + 1];
  __shared__ double di[NB];
  const int t = threadIdx.x;
  const double* L = L_base + blockIdx.z * sL + r0 * ldl + r0;
  const int64_t c0 = (int64_t)blockIdx.x * NB;
  const double* Y = Y_base + blockIdx.z * sY + r0 * ldy + c0;
  double* G = G_base + blockIdx.z * sG + r0 * ldg + c0;
  const bool colok = c0 + t < ncol;
  for (int r = 0; r < NB; ++r) {
    Ls[r][t] = (r < b && t < b) ? (t <= r ? L[r * ldl + t] : 0.0) : (r == t ? 1.0 : 0.0);
    Xs[r][t] = (r < b && colok) ? Y[r * ldy + t] : 0.0;
  }
  di[t] = t < b ? dinv_base[blockIdx.z * sD + r0 + t] : 1.0;
  __syncthreads();
  double x[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) x[q] = Xs[q][t];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const double xj = x[j] * di[j];
    x[j] = xj;
#pragma unroll
    for (int i = j + 1; i < NB; ++i) x[i] = fma(-Ls[i][j], xj, x[i]);
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) Xs[q][t] = x[q];
  __syncthreads();
  if (colok)
    for (int r = 0; r < b; ++r) G[r * ldg + t] = Xs[r][t];
}

}  // namespace

hipError_t potrf_f64(double* A, int64_t n, int64_t lda, int64_t sA, int batch, double* dinv,
                     int64_t sD, double* ldpart, int64_t sL, int* fail, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = batch > 0 ? batch : 1;
  for (int64_t c = 0; c < n; c += OUTER) {
    const int64_t pe = (c + OUTER < n) ? c + OUTER : n;
    for (int64_t q = c; q < pe; q += NB) {
      const int b = (int)((n - q) < NB ? (n - q) : NB);
      hipLaunchKernelGGL(k_potrf_diag, dim3(1, 1, nb), dim3(256), 0, s, A, lda, sA, q, b, dinv, sD,
                         ldpart, sL, (int)(q / NB), fail);
      CF_HIP_TRY(hipGetLastError());
      const int64_t below = n - (q + b);
      if (below <= 0) continue;
      hipLaunchKernelGGL(k_trsm_rows, dim3((unsigned)((below + NB - 1) / NB), 1, nb), dim3(64), 0, s,
                         A, lda, sA, q, b, below, dinv, sD);
      CF_HIP_TRY(hipGetLastError());
      if (q + b < pe) {   // rest of the outer panel
        GemmDesc g{};
        g.M = below; g.N = pe - (q + b); g.K = b;
        g.A = A + (q + b) * lda + q; g.lda = lda; g.at = 0;
        g.B = A + (q + b) * lda + q; g.ldb = lda; g.bt = 1;
        g.C = A + (q + b) * lda + (q + b); g.ldc = lda;
        g.alpha = -1.0; g.beta = 1.0; g.lower = 1;
        g.batch = nb; g.sA = sA; g.sB = sA; g.sC = sA;
        CF_HIP_TRY(gemm_f64(g, s));
      }
    }
    if (pe < n) {           // trailing matrix
      GemmDesc g{};
      g.M = n - pe; g.N = n - pe; g.K = pe - c;
      g.A = A + pe * lda + c; g.lda = lda; g.at = 0;
      g.B = A + pe * lda + c; g.ldb = lda; g.bt = 1;
      g.C = A + pe * lda + pe; g.ldc = lda;
      g.alpha = -1.0; g.beta = 1.0; g.lower = 1;
      g.batch = nb; g.sA = sA; g.sB = sA; g.sC = sA;
      CF_HIP_TRY(gemm_f64(g, s));
    }
  }
  return hipSuccess;
}

namespace {
hipError_t trsm_rec(const double* L, int64_t ldl, int64_t sL, const double* dinv, int64_t sD,
                    double* Y, int64_t ldy, int64_t sY, double* G, int64_t ldg, int64_t sG,
                    int64_t ncol, int64_t r0, int64_t r1, int batch, hipStream_t s) {
  if (r1 - r0 <= NB) {
    hipLaunchKernelGGL(k_trsm_cols, dim3((unsigned)((ncol + NB - 1) / NB), 1, batch), dim3(64), 0, s,
                       L, ldl, sL, dinv, sD, r0, (int)(r1 - r0), Y, ldy, sY, G, ldg, sG, ncol);
    return hipGetLastError();
  }
  int64_t nblk = (r1 - r0 + NB - 1) / NB;
  int64_t mid = r0 + ((nblk + 1) / 2) * NB;
  CF_HIP_TRY(trsm_rec(L, ldl, sL, dinv, sD, Y, ldy, sY, G, ldg, sG, ncol, r0, mid, batch, s));
  GemmDesc g{};
  g.M = r1 - mid; g.N = ncol; g.K = mid - r0;
  g.A = L + mid * ldl + r0; g.lda = ldl; g.at = 0;
  g.B = G + r0 * ldg; g.ldb = ldg; g.bt = 0;
  g.C = Y + mid * ldy; g.ldc = ldy;
  g.alpha = -1.0; g.beta = 1.0; g.lower = 0;
  g.batch = batch; g.sA = sL; g.sB = sG; g.sC = sY;
  CF_HIP_TRY(gemm_f64(g, s));
  return trsm_rec(L, ldl, sL, dinv, sD, Y, ldy, sY, G, ldg, sG, ncol, mid, r1, batch, s);
}
}  // namespace

hipError_t trsm_lower_f64(const double* L, int64_t n, int64_t ldl, int64_t sL, const double* dinv,
                          int64_t sD, double* Y, int64_t ldy, int64_t sY, double* G, int64_t ldg,
                          int64_t sG, int64_t ncol, int64_t r0, int batch, hipStream_t s) {
  if (ncol <= 0 || n <= 0) return hipSuccess;
  int64_t start = (r0 / NB) * NB;
  return trsm_rec(L, ldl, sL, dinv, sD, Y, ldy, sY, G, ldg, sG, ncol, start, n,
                  batch > 0 ? batch : 1, s);
}

}  // namespace cf
