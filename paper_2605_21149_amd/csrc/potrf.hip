// Blocked Cholesky C = L L^T, ln|C| from its diagonal, and forward substitution L^-1 Y.
//
// Right-looking, two-level blocking: 256-column outer panels whose 64-column diagonal blocks are
// factorised and inverted by one workgroup; the column panel below each block is then a GEMM
// with the inverted block (X L11^-T), and the remaining columns of the outer panel and the whole
// trailing matrix are updated with the same FP64 matrix-core GEMM.  The forward substitution
// L^-1 Y recurses on halves of the row range: leaves multiply by the inverted 64 x 64 diagonal
// block, interior nodes are GEMM updates.  Every flop outside the 64 x 64 blocks runs on MFMA.
#include "cf_internal.h"
#include <climits>

namespace cf {
namespace {

constexpr int NB = kNB;          // 64
constexpr int OUTER = 256;       // outer panel width

// Factor the b x b (b <= 64) diagonal block at (c, c) and invert the factor.
// 256 threads in a 16 x 16 grid; thread (ty, tx) keeps the 4 x 4 sub-block rows 4ty.., columns
// 4tx.. in registers.  Column j of the right-looking factorisation is published through LDS
// (double-buffered, one barrier per column) and applied as a rank-1 update with the unscaled
// column, a_rq -= a_rj a_qj / a_jj.  The inverse X = L^-1 then follows by the same scheme, row k
// of X and column k of L published per step.  Rows and columns beyond b are padded with the
// identity.  Outputs: L11 (lower) in place, L11^-1 as a full 64 x 64 block, the block's
// sum of ln L_jj, and the first non-positive pivot.
__global__ __launch_bounds__(256) void k_potrf_diag(double* A_base, int64_t lda, int64_t sA, int64_t c,
                                                    int b, double* Li_base, int64_t sLi,
                                                    double* ldpart_base, int64_t sL, int blk,
                                                    int* fail) {
  __shared__ double colb[2][NB];
  __shared__ double rowb[2][NB];
  __shared__ double piv[NB];
  __shared__ double rsq[NB];
  __shared__ double lg[NB];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double* A = A_base + blockIdx.z * sA + c * lda + c;
  double a[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * ty + i, q = 4 * tx + j;
      a[i][j] = (r < b && q < b) ? (q <= r ? A[r * lda + q] : 0.0) : (r == q ? 1.0 : 0.0);
    }
  // ---- factorisation; the masks (row > j, column > j) are applied as factors, not branches
  for (int j4 = 0; j4 < NB; j4 += 4) {
#pragma unroll
    for (int jj0 = 0; jj0 < 4; ++jj0) {
      const int j = j4 + jj0, buf = j & 1;
      if (tx == (j4 >> 2)) {
#pragma unroll
        for (int i = 0; i < 4; ++i) colb[buf][4 * ty + i] = a[i][jj0];
      }
      __syncthreads();
      const double d = colb[buf][j];
      if (tid == 0) piv[j] = d;
      const double inv = 1.0 / d;
      double cr[4], cq[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        cr[i] = (4 * ty + i > j) ? colb[buf][4 * ty + i] * inv : 0.0;
        cq[i] = (4 * tx + i > j) ? colb[buf][4 * tx + i] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) a[i][jj] = fma(-cr[i], cq[jj], a[i][jj]);
    }
  }
  __syncthreads();
  if (tid < NB) {
    const double d = piv[tid];
    rsq[tid] = 1.0 / sqrt(d);
    lg[tid] = (tid < b) ? 0.5 * log(d) : 0.0;
  }
  __syncthreads();
  // ---- scale to L and write it back
  double l[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int r = 4 * ty + i, q = 4 * tx + jj;
      l[i][jj] = (q < r) ? a[i][jj] * rsq[q] : (q == r ? sqrt(piv[q]) : 0.0);
      if (r < b && q < b && q <= r) A[r * lda + q] = l[i][jj];
    }
  // ---- X = L^-1 (right-looking forward substitution on the identity)
  double x[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) x[i][jj] = (4 * ty + i == 4 * tx + jj) ? 1.0 : 0.0;
  for (int k4 = 0; k4 < NB; k4 += 4) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = k4 + kk, buf = k & 1;
      if (ty == (k4 >> 2)) {
        const double dk = rsq[k];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          x[kk][jj] *= dk;
          rowb[buf][4 * tx + jj] = x[kk][jj];
        }
      }
      if (tx == (k4 >> 2)) {
#pragma unroll
        for (int i = 0; i < 4; ++i) colb[buf][4 * ty + i] = l[i][kk];
      }
      __syncthreads();
      double lr[4], xk[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        lr[i] = (4 * ty + i > k) ? colb[buf][4 * ty + i] : 0.0;
        xk[i] = rowb[buf][4 * tx + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) x[i][jj] = fma(-lr[i], xk[jj], x[i][jj]);
    }
  }
  double* Li = Li_base + blockIdx.z * sLi + (int64_t)blk * NB * NB;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) Li[(4 * ty + i) * NB + 4 * tx + jj] = x[i][jj];
  if (tid == 0) {
    // fixed-order sum of the block's ln L_jj; first non-positive pivot
    double acc = 0.0;
    int bad = INT_MAX;
    for (int j = 0; j < b; ++j) {
      const double d = piv[j];
      if (bad == INT_MAX && (!(d > 0.0) || !isfinite(d))) bad = (int)c + j;
      acc += lg[j];
    }
    ldpart_base[blockIdx.z * sL + blk] = acc;
    if (bad != INT_MAX) atomicMin(fail, bad);
  }
}

}  // namespace

hipError_t potrf_f64(double* A, int64_t n, int64_t lda, int64_t sA, int batch, double* Linv,
                     int64_t sLi, double* ldpart, int64_t sL, int* fail, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = batch > 0 ? batch : 1;
  for (int64_t c = 0; c < n; c += OUTER) {
    const int64_t pe = (c + OUTER < n) ? c + OUTER : n;
    for (int64_t q = c; q < pe; q += NB) {
      const int b = (int)((n - q) < NB ? (n - q) : NB);
      const int blk = (int)(q / NB);
      hipLaunchKernelGGL(k_potrf_diag, dim3(1, 1, nb), dim3(256), 0, s, A, lda, sA, q, b, Linv, sLi,
                         ldpart, sL, blk, fail);
      CF_HIP_TRY(hipGetLastError());
      const int64_t below = n - (q + b);
      if (below <= 0) continue;
      {   // column panel below the block: X <- X L11^-T, in place (each tile owns its rows)
        GemmDesc g{};
        g.M = below; g.N = b; g.K = b;
        g.A = A + (q + b) * lda + q; g.lda = lda; g.at = 0;
        g.B = Linv + (int64_t)blk * NB * NB; g.ldb = NB; g.bt = 1;
        g.C = A + (q + b) * lda + q; g.ldc = lda;
        g.alpha = 1.0; g.beta = 0.0; g.lower = 0;
        g.batch = nb; g.sA = sA; g.sB = sLi; g.sC = sA;
        CF_HIP_TRY(gemm_f64(g, s));
      }
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
// Leaves: G[r0:r0+b] = L11^-1 Y[r0:r0+b] (GEMM with the inverted diagonal block); interior
// nodes: Y[mid:r1] -= L[mid:r1, r0:mid] G[r0:mid].
hipError_t trsm_rec(const double* L, int64_t ldl, int64_t sL, const double* Linv, int64_t sLi,
                    double* Y, int64_t ldy, int64_t sY, double* G, int64_t ldg, int64_t sG,
                    int64_t ncol, int64_t r0, int64_t r1, int batch, hipStream_t s) {
  if (r1 - r0 <= NB) {
    GemmDesc g{};
    g.M = r1 - r0; g.N = ncol; g.K = r1 - r0;
    g.A = Linv + (r0 / NB) * NB * NB; g.lda = NB; g.at = 0;
    g.B = Y + r0 * ldy; g.ldb = ldy; g.bt = 0;
    g.C = G + r0 * ldg; g.ldc = ldg;
    g.alpha = 1.0; g.beta = 0.0; g.lower = 0;
    g.batch = batch; g.sA = sLi; g.sB = sY; g.sC = sG;
    return gemm_f64(g, s);
  }
  int64_t nblk = (r1 - r0 + NB - 1) / NB;
  int64_t mid = r0 + ((nblk + 1) / 2) * NB;
  CF_HIP_TRY(trsm_rec(L, ldl, sL, Linv, sLi, Y, ldy, sY, G, ldg, sG, ncol, r0, mid, batch, s));
  GemmDesc g{};
  g.M = r1 - mid; g.N = ncol; g.K = mid - r0;
  g.A = L + mid * ldl + r0; g.lda = ldl; g.at = 0;
  g.B = G + r0 * ldg; g.ldb = ldg; g.bt = 0;
  g.C = Y + mid * ldy; g.ldc = ldy;
  g.alpha = -1.0; g.beta = 1.0; g.lower = 0;
  g.batch = batch; g.sA = sL; g.sB = sG; g.sC = sY;
  CF_HIP_TRY(gemm_f64(g, s));
  return trsm_rec(L, ldl, sL, Linv, sLi, Y, ldy, sY, G, ldg, sG, ncol, mid, r1, batch, s);
}
}  // namespace

hipError_t trsm_lower_f64(const double* L, int64_t n, int64_t ldl, int64_t sL, const double* Linv,
                          int64_t sLi, double* Y, int64_t ldy, int64_t sY, double* G, int64_t ldg,
                          int64_t sG, int64_t ncol, int64_t r0, int batch, hipStream_t s) {
  if (ncol <= 0 || n <= 0) return hipSuccess;
  int64_t start = (r0 / NB) * NB;
  return trsm_rec(L, ldl, sL, Linv, sLi, Y, ldy, sY, G, ldg, sG, ncol, start, n,
                  batch > 0 ? batch : 1, s);
}

}  // namespace cf
