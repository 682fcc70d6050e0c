// Blocked Cholesky C = L L^T, ln|C| from its diagonal, and forward substitution L^-1 Y.
// Rows appended below C ride along the factorisation and come out as their forward solves.
//
// Right-looking, two-level blocking: 256-column outer panels whose 64-column diagonal blocks are
// factorised and inverted by one workgroup; the column panel below each block is then a GEMM
// with the inverted block (X L11^-T), and the remaining columns of the outer panel and the whole
// trailing matrix are updated with the same FP64 matrix-core GEMM.  The forward substitution
// L^-1 Y recurses on halves of the row range: leaves multiply by the inverted 64 x 64 diagonal
// block, interior nodes are GEMM updates.  Every flop outside the 64 x 64 blocks runs on MFMA.
#include "cf_internal.h"
#include <functional>

#include <climits>

namespace cf {
namespace {

constexpr int NB = kNB;          // 64
constexpr int OUTER = 256;       // width of the blocks whose inverses serve the triangular solves

// Factor the b x b (b <= 64) diagonal block at (c, c) and invert the factor in the same sweep.
// 256 threads on a 16 x 16 grid; thread (ty, tx) keeps the 4 x 4 sub-blocks (rows 4ty.., columns
// 4tx..) of the matrix and of X = L^-1 in registers.  The sweep runs over 4-column groups J:
//   A  thread (J, J) factors its 4 x 4 diagonal block and inverts it (register-local);
//   B  the threads of column group J form L_RJ = A_RJ L_JJ^-T for the rows below, the threads of
//      row group J form the finished rows X_J = L_JJ^-1 X_J; both are published through LDS;
//   C  every thread below applies the rank-4 updates A_RQ -= L_RJ L_QJ^T and X_R -= L_RJ X_J.
// Two barriers per 4 columns.  Reciprocal square roots use the hardware estimate refined by
// Newton steps.  Rows and columns beyond b are padded with the identity.  Outputs: L11 (lower)
// in place, L11^-1 as a full 64 x 64 block, the block's sum of ln L_jj and the first
// non-positive pivot.
__device__ __forceinline__ double rsq_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * fma(-0.5 * d * y, y, 1.5);
  return y * fma(-0.5 * d * y, y, 1.5);
}

__global__ __launch_bounds__(256) void k_potrf_diag(double* A_base, int64_t lda, int64_t sA, int64_t c,
                                                    int b, double* Li_base, int64_t sLi,
                                                    double* ldpart_base, int64_t sL, int blk,
                                                    int* fail) {
  __shared__ double Ljji[2][16];          // L_JJ^-1 (4 x 4, row-major)
  __shared__ double colblk[2][NB][4];     // L_RJ, all rows
  __shared__ double rowblk[2][4][NB];     // X_J, all columns
  __shared__ double prodp[16];
  __shared__ int badp[16];
  // the diagonal blocks are the head of the critical chain: their waves win SIMD issue over the
  // bulk update waves that share the CU
  __builtin_amdgcn_s_setprio(2);
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double* A = A_base + blockIdx.z * sA + c * lda + c;
  double a[4][4], x[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * ty + i, q = 4 * tx + j;
      a[i][j] = (r < b && q < b) ? (q <= r ? A[r * lda + q] : 0.0) : (r == q ? 1.0 : 0.0);
      x[i][j] = (r == q) ? 1.0 : 0.0;
    }
  for (int J = 0; J < 16; ++J) {
    const int buf = J & 1;
    // ---- A: the 4 x 4 diagonal block
    if (tx == J && ty == J) {
      double l[4][4], y[4];
      double prod = 1.0;
      int bad = INT_MAX;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        double d = a[cc][cc];
#pragma unroll
        for (int k = 0; k < cc; ++k) d = fma(-l[cc][k], l[cc][k], d);
        if (bad == INT_MAX && (!(d > 0.0) || !isfinite(d)) && 4 * J + cc < b) bad = (int)c + 4 * J + cc;
        prod *= d;
        y[cc] = rsq_nr(d);
        l[cc][cc] = d * y[cc];
#pragma unroll
        for (int r = cc + 1; r < 4; ++r) {
          double t = a[r][cc];
#pragma unroll
          for (int k = 0; k < cc; ++k) t = fma(-l[r][k], l[cc][k], t);
          l[r][cc] = t * y[cc];
        }
#pragma unroll
        for (int r = 0; r < cc; ++r) l[r][cc] = 0.0;
      }
      // inverse of the 4 x 4 lower factor
      double li[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) li[i][j] = 0.0;
        li[i][i] = y[i];
#pragma unroll
        for (int j = 0; j < i; ++j) {
          double t = 0.0;
#pragma unroll
          for (int k = j; k < i; ++k) t = fma(l[i][k], li[k][j], t);
          li[i][j] = -t * y[i];
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          a[i][j] = l[i][j];
          Ljji[buf][i * 4 + j] = li[i][j];
        }
      prodp[J] = prod;                       // logarithms are taken after the sweep
      badp[J] = bad;
    }
    __syncthreads();
    // ---- B: column group J below the diagonal, row group J of X
    double li[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) li[i][j] = Ljji[buf][i * 4 + j];
    if (tx == J && ty > J) {
      double l[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          double t = 0.0;
#pragma unroll
          for (int k = 0; k <= cc; ++k) t = fma(a[i][k], li[cc][k], t);   // (A L^-T)[i][cc]
          l[i][cc] = t;
        }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          a[i][cc] = l[i][cc];
          colblk[buf][4 * ty + i][cc] = l[i][cc];
        }
    }
    if (ty == J && tx <= J) {          // X_J vanishes right of column group J
      double xn[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          double t = 0.0;
#pragma unroll
          for (int k = 0; k <= i; ++k) t = fma(li[i][k], x[k][jj], t);
          xn[i][jj] = t;
        }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          x[i][jj] = xn[i][jj];
          rowblk[buf][i][4 * tx + jj] = xn[i][jj];
        }
    }
    __syncthreads();
    // ---- C: rank-4 updates below.  Lanes right of the column group update the factor (only on or
    //      below the diagonal: J < tx <= ty), lanes left of it the inverse (X_J vanishes right of J:
    //      tx <= J); one shared FMA path with per-lane operands.
    if (ty > J && tx <= ty) {
      const bool inv = tx <= J;
      double lr[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) lr[i][cc] = colblk[buf][4 * ty + i][cc];
      double w[4][4];                  // w[cc][jj]: X_J[cc][4tx+jj] or L_QJ[4tx+jj][cc]
#pragma unroll
      for (int cc = 0; cc < 4; ++cc)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          w[cc][jj] = inv ? rowblk[buf][cc][4 * tx + jj] : colblk[buf][4 * tx + jj][cc];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          double t = inv ? x[i][jj] : a[i][jj];
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) t = fma(-lr[i][cc], w[cc][jj], t);
          if (inv) x[i][jj] = t; else a[i][jj] = t;
        }
    }
  }
  // ---- write L (lower), L^-1, log det part, first bad pivot
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int r = 4 * ty + i, q = 4 * tx + jj;
      if (r < b && q < b && q <= r) A[r * lda + q] = a[i][jj];
    }
  double* Li = Li_base + blockIdx.z * sLi + (int64_t)blk * NB * NB;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) Li[(4 * ty + i) * NB + 4 * tx + jj] = x[i][jj];
  __syncthreads();
  if (tid < 16) prodp[tid] = 0.5 * log(prodp[tid]);
  __syncthreads();
  if (tid == 0) {
    double acc = 0.0;
    int bad = INT_MAX;
    for (int J = 0; J < 16; ++J) {
      acc += prodp[J];
      if (bad == INT_MAX && badp[J] != INT_MAX) bad = badp[J];
    }
    ldpart_base[blockIdx.z * sL + blk] = acc;
    if (bad != INT_MAX) atomicMin(fail, bad);
  }
}

// The same for batches of factorisations, with a shorter dependent chain.  256 threads, four
// waves; lane r of wave w holds row r of the block's columns 16w..16w+15 in registers.
//   1. Column sweep.  Wave w first applies the updates of the columns left of its own as the
//      waves owning them announce them (the column in LDS plus a ready flag, no barrier), then
//      factors its 16 columns.  From one pivot to the next the chain is the reciprocal square root
//      and d_(j+1) = p - (q y_j)^2 with p, q (entries of lane j + 1) read beforehand; the next two
//      columns take column j's update at once, the others during the next chain.
//   2. Inverse X = L^-1 by blocks of 16: each wave inverts its diagonal block by substitution
//      (one column of X per lane), then the off-diagonal blocks follow from
//      [A 0; B C]^-1 = [A^-1 0; -C^-1 B A^-1  C^-1] at 32 and at 64 columns, as FP64 matrix-core
//      products (one 16 x 16 output tile per wave).
// Outputs as k_potrf_diag.  Measured on blocks of n = 5952: 23-27 us against 31-34 us, and a
// batch of 8 likelihood points 16.2 -> 15.7 ms; a single factorisation, whose chain runs on a few
// reserved CUs, became slower with it (12.2 -> 12.3 ms for Fisher + QML) and keeps k_potrf_diag.
// The waits on the ready flags are bounded; a wait that runs out (which needs a fault elsewhere)
// reports the block's first column as a failed pivot instead of hanging.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Waits until another wave of the workgroup sets *f; false after about 2^20 polls.
__device__ __forceinline__ bool wait_flag(const int* f) {
  for (int i = 0; i < (1 << 20); ++i) {
    if (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) return true;
    __builtin_amdgcn_s_sleep(1);
  }
  return false;
}

typedef double dbl4d __attribute__((ext_vector_type(4)));

// Offset of column j in a 64 x 64 lower triangle packed by columns (entry i >= j at PK(j) + i).
__device__ __forceinline__ int PK(int j) { return j * NB - (j * (j + 1)) / 2; }

__global__ __launch_bounds__(256) void k_potrf_diag_sweep(double* A_base, int64_t lda, int64_t sA, int64_t c,
                                                    int b, double* Li_base, int64_t sLi,
                                                    double* ldpart_base, int64_t sL, int blk,
                                                    int* fail) {
  constexpr int LS = NB + 1;               // row stride of X in LDS
  constexpr int TS = 33;                   // row stride of the 32 x 32 product buffer
  // L by columns, lower triangle packed: L_ij (i >= j) at colP[PK(j) + i]; the space holds the
  // 32 x 32 product of the last inverse step once L is no longer read.  52 KB in all (76 KB
  // unpacked, which measured slower in the batched factorisation).
  // (the 64 entries past the triangle take the stores of the lanes above the diagonal)
  constexpr int PSZ = NB * (NB + 1) / 2;
  __shared__ double colP[PSZ + 64];
  __shared__ double Xs[NB * LS];           // X = L^-1, row-major
  __shared__ double yv[NB], dv[NB];        // 1 / L_jj and the pivots
  __shared__ int ready[NB + 64];           // flags; the 64 past NB take the other lanes' stores
  __shared__ int stall;
  // the diagonal blocks are the head of the critical chain: their waves win SIMD issue over the
  // bulk update waves that share the CU
  __builtin_amdgcn_s_setprio(2);
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (tid < NB) ready[tid] = 0;
  if (tid == 0) stall = 0;
  for (int i = tid; i < NB * LS; i += 256) Xs[i] = 0.0;
  double* A = A_base + blockIdx.z * sA + c * lda + c;
  double a[16];
#pragma unroll
  for (int cc = 0; cc < 16; ++cc) {
    const int q = 16 * w + cc;
    a[cc] = (lane < b && q < b) ? (q <= lane ? A[lane * lda + q] : 0.0) : (lane == q ? 1.0 : 0.0);
  }
  __syncthreads();
  // ---- 1a. updates from the columns left of this wave's, as they are published
  bool ok = true;
  for (int j = 0; j < 16 * w; ++j) {
    ok = wait_flag(&ready[j]) && ok;
    const double lv = colP[PK(j) + (lane >= j ? lane : j)];
    const double l = lane >= j ? lv : 0.0;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) a[cc] = fma(-l, colP[PK(j) + 16 * w + cc], a[cc]);
  }
  // ---- 1b. this wave's columns.  The chain from one pivot to the next is the reciprocal square
  //      root and d_(j+1) = p - (q y_j)^2, with p = A_(j+1,j+1) and q = A_(j+1,j) read beforehand
  //      (the value lane j + 1 then forms itself, up to rounding).  The next two columns take
  //      column j's update at once (their entries give the next p, q); the columns beyond take it
  //      from the column's LDS copy during the next chain.  Column j - 1 is announced after
  //      column j's chain; the flag and column stores are plain LDS stores, which the wave
  //      performs in order.
  double dj = readlane_f64(a[0], 16 * w);
  double my_y = 0.0, my_d = 0.0;           // lane j keeps 1 / L_jj and the pivot
#pragma unroll
  for (int jj = 0; jj < 16; ++jj) {
    const int j = 16 * w + jj;
    double q1 = 0.0, p1 = 0.0, r2 = 0.0;
    if (jj + 1 < 16) {
      q1 = readlane_f64(a[jj], j + 1);
      p1 = readlane_f64(a[jj + 1], j + 1);
    }
    if (jj + 2 < 16) r2 = readlane_f64(a[jj], j + 2);
    if (jj > 0) {                          // column j - 1 into the columns beyond the two it updated
      const double lp = a[jj - 1];
#pragma unroll
      for (int cc = jj + 2; cc < 16; ++cc) a[cc] = fma(-lp, colP[PK(j - 1) + 16 * w + cc], a[cc]);
    }
    // y = 1 / sqrt(d): hardware estimate, two Newton steps (the second's product formed early)
    const double y0 = __builtin_amdgcn_rsq(dj);
    const double h = -0.5 * dj;
    const double e = h * y0;
    const double f = fma(e, y0, 1.5);
    const double y1 = y0 * f;
    const double f2 = fma(e * f, y1, 1.5);
    const double y = y1 * f2;
    double lc = 0.0, dn = 0.0;
    if (jj + 1 < 16) {
      lc = (q1 * y1) * f2;                 // L_(j+1,j)
      dn = fma(-lc, lc, p1);               // the next pivot
    }
    const double l = lane > j ? a[jj] * y : (lane == j ? dj * y : 0.0);
    a[jj] = l;
    if (jj + 1 < 16) a[jj + 1] = fma(-l, lc, a[jj + 1]);
    if (jj + 2 < 16) a[jj + 2] = fma(-l, r2 * y, a[jj + 2]);
    my_y = lane == j ? y : my_y;
    my_d = lane == j ? dj : my_d;
    if (jj > 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __hip_atomic_store(&ready[lane == 0 ? j - 1 : NB + lane], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    colP[PSZ + lane + ((PK(j) - PSZ) & -(int)(lane >= j))] = l;   // (a select, kept branch-free)
    dj = dn;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __hip_atomic_store(&ready[lane == 0 ? 16 * w + 15 : NB + lane], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  if (lane >= 16 * w && lane < 16 * w + 16) {
    yv[lane] = my_y;
    dv[lane] = my_d;
  }
  if (!ok) stall = 1;
  // L (lower) in place
#pragma unroll
  for (int cc = 0; cc < 16; ++cc) {
    const int q = 16 * w + cc;
    if (lane < b && q < b && q <= lane) A[lane * lda + q] = a[cc];
  }
  __syncthreads();
  // ---- 2a. the diagonal 16-block of wave w: lane k < 16 forms column 16w + k of X
  if (lane < 16) {
    double s[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) s[r] = r == lane ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double xk = s[k] * yv[16 * w + k];
      Xs[(16 * w + k) * LS + 16 * w + lane] = xk;
#pragma unroll
      for (int r = k + 1; r < 16; ++r) s[r] = fma(-colP[PK(16 * w + k) + 16 * w + r], xk, s[r]);
    }
  }
  __syncthreads();
  // ---- 2b. the 16 x 16 blocks below the diagonal pairs: X_10 (wave 0) and X_32 (wave 1)
  //      X_{P+1,P} = -X_{P+1,P+1} (L_{P+1,P} X_{PP}); the first product's accumulator already holds
  //      the second one's B operand (row 4kq + lane/16, column lane%16 of slab kq)
  const int ri = lane & 15, rk = lane >> 4;
  if (w < 2) {
    const int p0 = 32 * w;
    dbl4d t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) {
      const int k = p0 + 4 * kq + rk;
      t = __builtin_amdgcn_mfma_f64_16x16x4f64(colP[PK(k) + p0 + 16 + ri], Xs[k * LS + p0 + ri], t, 0, 0, 0);
    }
    dbl4d o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kq = 0; kq < 4; ++kq)
      o = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[(p0 + 16 + ri) * LS + p0 + 16 + 4 * kq + rk], t[kq], o, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) Xs[(p0 + 16 + rk + 4 * r) * LS + p0 + ri] = -o[r];
  }
  __syncthreads();
  // ---- 2c. the 32 x 32 block X[32:64, 0:32] = -X[32:64, 32:64] (L[32:64, 0:32] X[0:32, 0:32]);
  //      wave w owns output tile (ta, tb) of both products
  const int ta = w >> 1, tb = w & 1;
  {
    dbl4d t = {0.0, 0.0, 0.0, 0.0};
    for (int kq = 4 * tb; kq < 8; ++kq) {            // X[k, 16tb..] vanishes for k < 16tb
      const int k = 4 * kq + rk;
      t = __builtin_amdgcn_mfma_f64_16x16x4f64(colP[PK(k) + 32 + 16 * ta + ri], Xs[k * LS + 16 * tb + ri], t, 0, 0, 0);
    }
    __syncthreads();                                  // L is read for the last time above
    double* Ts = colP;
#pragma unroll
    for (int r = 0; r < 4; ++r) Ts[(16 * ta + rk + 4 * r) * TS + 16 * tb + ri] = t[r];
  }
  __syncthreads();
  {
    dbl4d o = {0.0, 0.0, 0.0, 0.0};
    const double* Ts = colP;
    for (int kq = 0; kq < 4 * (ta + 1); ++kq) {       // X[32 + 16ta.., 32 + k] vanishes for k >= 16(ta + 1)
      const int k = 4 * kq + rk;
      o = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[(32 + 16 * ta + ri) * LS + 32 + k], Ts[k * TS + 16 * tb + ri], o,
                                               0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Xs[(32 + 16 * ta + rk + 4 * r) * LS + 16 * tb + ri] = -o[r];
  }
  __syncthreads();
  // ---- outputs: L^-1, the block's sum of ln L_jj = 1/2 ln d_j, the first non-positive pivot
  double* Li = Li_base + blockIdx.z * sLi + (int64_t)blk * NB * NB;
  for (int i = tid; i < NB * NB; i += 256) Li[i] = Xs[(i >> 6) * LS + (i & 63)];
  if (w == 0) {
    const double d = dv[lane];             // pivots of padded columns are 1
    const bool bad = lane < b && (!(d > 0.0) || !isfinite(d));
    const unsigned long long m = __ballot(bad);
    double v = lane < b ? 0.5 * log(d) : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) {
      ldpart_base[blockIdx.z * sL + blk] = v;
      if (m) atomicMin(fail, (int)c + (int)__builtin_ctzll(m));
      else if (stall) atomicMin(fail, (int)c);
    }
  }
}

__global__ void k_tri256_init(const double* Li64_base, int64_t sLi64, double* Li256_base, int64_t sLi256,
                              int p) {
  const double* Li64 = Li64_base + blockIdx.z * sLi64 + (int64_t)(4 * p) * NB * NB;
  double* D = Li256_base + blockIdx.z * sLi256 + (int64_t)p * 256 * 256;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < 256 * 256; idx += gridDim.x * blockDim.x) {
    const int r = idx >> 8, c = idx & 255;
    const int br = r >> 6, bc = c >> 6;
    D[idx] = (br == bc) ? Li64[(int64_t)br * NB * NB + (r & 63) * NB + (c & 63)] : 0.0;
  }
}

hipError_t gemm_plain(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, int64_t sA,
                      const double* B, int64_t ldb, int64_t sB, double* C, int64_t ldc, int64_t sC,
                      double alpha, int batch, hipStream_t s) {
  GemmDesc g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = 0.0; g.batch = batch; g.sA = sA; g.sB = sB; g.sC = sC;
  return gemm_f64(g, s);
}

// Inverse of the full 256 x 256 diagonal block of panel p from its 64-block inverses:
// [A 0; B C]^-1 = [A^-1 0; -C^-1 B A^-1  C^-1], applied at 128 and then at 256.
hipError_t tri256(const Factor& F, int p, double* scratch, hipStream_t s) {
  const int nb = F.batch;
  const int64_t c = (int64_t)p * 256, ld = F.ld;
  double* D = F.Li256 + (int64_t)p * 256 * 256;
  hipLaunchKernelGGL(k_tri256_init, dim3(64, 1, nb), dim3(256), 0, s, F.Li64, F.sLi64, F.Li256, F.sLi256, p);
  CF_HIP_TRY(hipGetLastError());
  const int64_t sS = 2 * 64 * 64 + 128 * 128;
  for (int h = 0; h < 2; ++h) {
    const int64_t o = c + 128 * h;
    const double* Bh = F.L + (o + 64) * ld + o;                        // L[o+64 : o+128, o : o+64]
    const double* Ainv = D + (128 * h) * 256 + 128 * h;                // 64 x 64 at (128h, 128h)
    const double* Cinv = D + (128 * h + 64) * 256 + 128 * h + 64;      // at (128h+64, 128h+64)
    double* T = scratch + h * 64 * 64;
    CF_HIP_TRY(gemm_plain(64, 64, 64, Bh, ld, F.sL, Ainv, 256, F.sLi256, T, 64, sS, 1.0, nb, s));
    CF_HIP_TRY(gemm_plain(64, 64, 64, Cinv, 256, F.sLi256, T, 64, sS, D + (128 * h + 64) * 256 + 128 * h,
                          256, F.sLi256, -1.0, nb, s));
  }
  const double* B2 = F.L + (c + 128) * ld + c;                         // L[c+128 : c+256, c : c+128]
  double* T = scratch + 2 * 64 * 64;
  CF_HIP_TRY(gemm_plain(128, 128, 128, B2, ld, F.sL, D, 256, F.sLi256, T, 128, sS, 1.0, nb, s));
  CF_HIP_TRY(gemm_plain(128, 128, 128, D + 128 * 256 + 128, 256, F.sLi256, T, 128, sS, D + 128 * 256, 256,
                        F.sLi256, -1.0, nb, s));
  return hipSuccess;
}

GemmDesc upd(const Factor& F, int64_t r0, int64_t c0, int64_t M, int64_t N, int64_t k0, int64_t K,
             int prio = 0) {
  // C[r0.., c0..] -= L[r0.., k0..k0+K] L[c0.., k0..k0+K]^T  (lower tiles relative to the diagonal)
  GemmDesc g{};
  g.M = M; g.N = N; g.K = K;
  g.A = F.L + r0 * F.ld + k0; g.lda = F.ld; g.at = 0;
  g.B = F.L + c0 * F.ld + k0; g.ldb = F.ld; g.bt = 1;
  g.C = F.L + r0 * F.ld + c0; g.ldc = F.ld;
  g.alpha = -1.0; g.beta = 1.0; g.lower = 1; g.diag_off = c0 - r0;
  g.batch = F.batch; g.sA = F.sL; g.sB = F.sL; g.sC = F.sL;
  g.mode = F.mode;
  g.tile = F.tile;
  g.tag = 2;                     // its own kernel instance in FP64 (ignored by the mixed modes)
  g.prio = prio;
  return g;
}

// X[:, c0..c1) -= X[:, k0..k1) L[c0..c1, k0..k1)^T for the rx extra rows X (ld F.ld).
GemmDesc xupd(const Factor& F, double* X, int64_t rx, int64_t k0, int64_t k1, int64_t c0, int64_t c1) {
  GemmDesc u{};
  u.M = rx; u.N = c1 - c0; u.K = k1 - k0;
  u.A = X + k0; u.lda = F.ld; u.at = 0;
  u.B = F.L + c0 * F.ld + k0; u.ldb = F.ld; u.bt = 1;
  u.C = X + c0; u.ldc = F.ld;
  u.alpha = -1.0; u.beta = 1.0;
  u.batch = F.batch; u.sA = F.sL; u.sB = F.sL; u.sC = F.sL;
  u.mode = F.mode;
  u.tile = F.tile;
  return u;
}

// Extra-row updates wait until the pending panels span kDefer columns.  Measured with the host
// paced one panel ahead (n = 5952 with 6965 extra rows, 256-column panels): 256 (every panel at
// once) 11.8 ms for Fisher + QML, 512 12.0-12.1, 1024 13.1, 2048 13.7.
constexpr int64_t kDefer = 256;

}  // namespace

hipError_t potrf_f64(Factor& F, double* scratch, const Streams& st) {
  const int64_t n = F.n, lda = F.ld;
  if (n <= 0) return hipSuccess;
  const unsigned nb = F.batch > 0 ? F.batch : 1;
  hipStream_t s = st.s;
  // All three roles on one stream (a caller that creates no streams or events): stream order
  // already serialises everything, so no event is recorded or waited on.
  const bool one = st.s1 == s && st.s2 == s;
  auto erec = [&](hipEvent_t e, hipStream_t on) { return one ? hipSuccess : hipEventRecord(e, on); };
  auto ewait = [&](hipStream_t on, hipEvent_t e) { return one ? hipSuccess : hipStreamWaitEvent(on, e, 0); };
  bool pending_b = false, pending_i = false;
  int64_t px = 0;                            // first panel column whose extra-row update is pending
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  CF_HIP_TRY(hipStreamIsCapturing(s, &cap));
  const bool capturing = cap != hipStreamCaptureStatusNone;
  // Outer panel width: a single factorisation is bound by its chain of diagonal blocks and keeps
  // 256-column panels; a batch is bound by its trailing updates, which run markedly faster as
  // rank-512 products (the C tile is read and written half as often per flop).
  const int64_t W = F.panel > 0 ? F.panel : (nb > 1 ? 512 : 256);
  const int64_t rows = F.rows > n ? F.rows : n;
  auto rows_for = [&](int64_t pe) { return (F.rows_early > 0 && pe <= F.p_early) ? F.rows_early : rows; };
  double* X = F.L + n * lda;                 // extra rows
  // A batch folds its extra rows into the rows of the panel solves and the updates (they follow
  // the matrix rows in memory) instead of solving them apart on the side stream: measured on a
  // batch of 8 at n = 5952 with 64 maps, factorisation 16.4 -> 15.9 ms; the QU N_side 16 scan
  // 1777 -> 1805 points/s.  A single factorisation, whose thousands of solve rows fill the bulk
  // CUs beside a chain on reserved ones, keeps them apart.
  const bool fold = nb > 1 && rows > n && F.rows_early == 0;
  const int64_t nr = fold ? rows : n;        // rows of the panel solves and updates
  // One 64-column block: factor and invert the diagonal block, then X <- X L11^-T for the column
  // panel below it (in place; each tile owns its rows).
  auto block = [&](int64_t q) -> hipError_t {
    const int b = (int)((n - q) < NB ? (n - q) : NB);
    const int blk = (int)(q / NB);
    hipLaunchKernelGGL(nb > 1 ? k_potrf_diag_sweep : k_potrf_diag, dim3(1, 1, nb), dim3(256), 0, s, F.L, lda, F.sL, q, b, F.Li64,
                       F.sLi64, F.ldpart, F.sPart, blk, F.fail);
    CF_HIP_TRY(hipGetLastError());
    const int64_t below = nr - (q + b);
    if (below <= 0) return hipSuccess;
    GemmDesc g{};
    g.M = below; g.N = b; g.K = b;
    g.A = F.L + (q + b) * lda + q; g.lda = lda; g.at = 0;
    g.B = F.Li64 + (int64_t)blk * NB * NB; g.ldb = NB; g.bt = 1;
    g.C = F.L + (q + b) * lda + q; g.ldc = lda;
    g.alpha = 1.0; g.beta = 0.0; g.lower = 0;
    g.batch = nb; g.sA = F.sL; g.sB = F.sLi64; g.sC = F.sL;
    g.prio = 2;
    return gemm_f64(g, s);
  };
  // Right-looking panel: after each block, a rank-64 update of the panel's remaining columns.
  // Each launch is short (K = 64), which suits a single factorisation whose launches fill only
  // part of the chip and whose chain is bound by launch latency.
  auto panel_right = [&](int64_t c0, int64_t c1) -> hipError_t {
    for (int64_t q = c0; q < c1; q += NB) {
      CF_HIP_TRY(block(q));
      const int64_t qe = q + NB;
      if (qe < c1) CF_HIP_TRY(gemm_f64(upd(F, qe, qe, nr - qe, c1 - qe, q, NB, 2), s));
    }
    return hipSuccess;
  };
  // Recursive panel: factor the left half, update the right half with one product of rank equal
  // to the left half's width, factor the right half.  The same flops as the right-looking order,
  // but half of them in rank-(W/2) products, which run several times faster per flop than rank-64
  // ones once a batch fills the chip.
  std::function<hipError_t(int64_t, int64_t)> panel_rec = [&](int64_t c0, int64_t c1) -> hipError_t {
    if (c1 - c0 <= NB) return block(c0);
    const int64_t nbk = (c1 - c0 + NB - 1) / NB;
    const int64_t mid = c0 + ((nbk + 1) / 2) * NB;
    CF_HIP_TRY(panel_rec(c0, mid));
    CF_HIP_TRY(gemm_f64(upd(F, mid, mid, nr - mid, c1 - mid, c0, mid - c0, 2), s));
    return panel_rec(mid, c1);
  };
  const bool rec = nb > 1;   // measured on batches of 8 at n = 5952: 20.0 -> 18.5 ms
  for (int64_t c = 0; c < n; c += W) {
    const int64_t pe = (c + W < n) ? c + W : n;
    // ---- critical path: the diagonal blocks and panels of this outer panel (rows of C only)
    CF_HIP_TRY(rec ? panel_rec(c, pe) : panel_right(c, pe));
    CF_HIP_TRY(erec(st.eL, s));
    // ---- keep the host at most one panel ahead of the device: the rest of this panel's launches
    //      are issued once the previous panel's chain has run.  Measured: with every panel of
    //      every stream queued up front, the device dispatches the critical chain markedly later
    //      (a single n = 5952 factorisation with its solves: 12.0 ms unthrottled, 10.0 ms two
    //      panels ahead, 9.2 ms one panel ahead; batches are indifferent between one and two).
    //      Graph capture records launches without running them, so it is never throttled.
    if (st.ring && !capturing) {
      const int64_t pidx = c / W;
      CF_HIP_TRY(hipEventRecord(st.ring[pidx % 4], s));
      if (pidx >= 1) CF_HIP_TRY(hipEventSynchronize(st.ring[(pidx - 1) % 4]));
    }
    // ---- 256-block inverse for the solves (side stream)
    if (F.Li256 && pe - c >= OUTER) {
      CF_HIP_TRY(ewait(st.s2, st.eL));
      for (int64_t q = c; q + OUTER <= pe; q += OUTER) CF_HIP_TRY(tri256(F, (int)(q / OUTER), scratch, st.s2));
      pending_i = true;
    }
    // ---- extra rows (side stream): solve against this panel, then pass the contributions of the
    //      pending panels [px, pe) on to the next panel's columns, and to all later columns once
    //      they span kDefer columns.  Extra rows never feed back into C, so they trail the
    //      factorisation.
    const int64_t rx = fold ? 0 : rows_for(pe) - n;
    const int64_t pn = (pe + W < n) ? pe + W : n;    // end of the next panel
    if (rx > 0) {
      CF_HIP_TRY(ewait(st.s2, st.eL));
      for (int64_t q = c; q < pe; q += NB) {
        const int b = (int)((n - q) < NB ? (n - q) : NB);
        GemmDesc g{};                                          // X_q <- X_q L_qq^-T (in place)
        g.M = rx; g.N = b; g.K = b;
        g.A = X + q; g.lda = lda; g.at = 0;
        g.B = F.Li64 + (q / NB) * NB * NB; g.ldb = NB; g.bt = 1;
        g.C = X + q; g.ldc = lda;
        g.alpha = 1.0; g.beta = 0.0;
        g.batch = nb; g.sA = F.sL; g.sB = F.sLi64; g.sC = F.sL;
        CF_HIP_TRY(gemm_f64(g, st.s2));
        if (q + b < pe) CF_HIP_TRY(gemm_f64(xupd(F, X, rx, q, q + b, q + b, pe), st.s2));
      }
      if (pe < n) {
        if (pe - px >= kDefer || pn >= n) {        // all pending panels into all later columns
          CF_HIP_TRY(gemm_f64(xupd(F, X, rx, px, pe, pe, n), st.s2));
          px = pe;
        } else {                                   // only into the next panel's columns
          CF_HIP_TRY(gemm_f64(xupd(F, X, rx, px, pe, pe, pn), st.s2));
        }
      }
      pending_i = true;
    }
    if (pe >= n) break;
    // ---- lookahead: the next panel's columns on the critical path, after the previous bulk update
    if (st.eA) {
      // on the bulk CUs, after the previous trailing update (stream order) and this panel's chain
      CF_HIP_TRY(ewait(st.s1, st.eL));
      CF_HIP_TRY(gemm_f64(upd(F, pe, pe, nr - pe, pn - pe, c, pe - c, 1), st.s1));
      CF_HIP_TRY(erec(st.eA, st.s1));
      CF_HIP_TRY(ewait(s, st.eA));
    } else {
      // after the previous trailing update, or with eT only after its first part: the columns of
      // this lookahead's panel (the rest of that update runs on beside the next panels' chains)
      if (pending_b) CF_HIP_TRY(ewait(s, st.eT ? st.eT : st.eB));
      CF_HIP_TRY(gemm_f64(upd(F, pe, pe, nr - pe, pn - pe, c, pe - c, 1), s));
    }
    // ---- bulk trailing update beyond the next panel (side stream, overlaps the next panel)
    if (pn < n) {
      CF_HIP_TRY(ewait(st.s1, st.eL));
      const int64_t pn2 = (pn + W < n) ? pn + W : n;    // end of the panel after next
      if (st.eT && !st.eA && pn2 < n) {
        CF_HIP_TRY(gemm_f64(upd(F, pn, pn, nr - pn, pn2 - pn, c, pe - c), st.s1));
        CF_HIP_TRY(erec(st.eT, st.s1));
        CF_HIP_TRY(gemm_f64(upd(F, pn2, pn2, nr - pn2, n - pn2, c, pe - c), st.s1));
      } else {
        CF_HIP_TRY(gemm_f64(upd(F, pn, pn, nr - pn, n - pn, c, pe - c), st.s1));
        if (st.eT && !st.eA) CF_HIP_TRY(erec(st.eT, st.s1));
      }
      CF_HIP_TRY(erec(st.eB, st.s1));
      pending_b = true;
    }
  }
  if (pending_b) CF_HIP_TRY(ewait(s, st.eB));
  if (pending_i) {
    CF_HIP_TRY(erec(st.eI, st.s2));
    CF_HIP_TRY(ewait(s, st.eI));
  }
  return hipSuccess;
}

namespace {
// Leaves multiply by an inverted diagonal block (256 rows when an aligned full 256-block inverse
// exists, else 64); interior nodes are GEMM updates Y[mid:r1] -= L[mid:r1, r0:mid] G[r0:mid].
hipError_t trsm_rec(const Factor& F, double* Y, int64_t ldy, int64_t sY, double* G, int64_t ldg,
                    int64_t sG, int64_t ncol, int64_t r0, int64_t r1, hipStream_t s) {
  const int batch = F.batch > 0 ? F.batch : 1;
  const bool leaf256 = F.Li256 && (r0 % 256) == 0 && r1 - r0 == 256;
  if (r1 - r0 <= NB || leaf256) {
    const int64_t m = r1 - r0;
    GemmDesc g{};
    g.M = m; g.N = ncol; g.K = m;
    if (leaf256) { g.A = F.Li256 + (r0 / 256) * 256 * 256; g.lda = 256; g.sA = F.sLi256; }
    else { g.A = F.Li64 + (r0 / NB) * NB * NB; g.lda = NB; g.sA = F.sLi64; }
    g.at = 0;
    g.B = Y + r0 * ldy; g.ldb = ldy; g.bt = 0;
    g.C = G + r0 * ldg; g.ldc = ldg;
    g.alpha = 1.0; g.beta = 0.0; g.lower = 0;
    g.batch = batch; g.sB = sY; g.sC = sG;
    g.mode = F.mode;
    return gemm_f64(g, s);
  }
  int64_t mid;
  const int64_t up = ((r0 + 255) / 256) * 256;
  if (F.Li256 && r0 % 256 != 0 && up < r1) {
    mid = up;                                    // reach a 256-aligned row first
  } else if (F.Li256 && r0 % 256 == 0 && r1 - r0 > 256) {
    const int64_t n256 = (r1 - r0 + 255) / 256;
    mid = r0 + ((n256 + 1) / 2) * 256;
    if (mid >= r1) mid = r0 + 256;
  } else {
    const int64_t nblk = (r1 - r0 + NB - 1) / NB;
    mid = r0 + ((nblk + 1) / 2) * NB;
  }
  CF_HIP_TRY(trsm_rec(F, Y, ldy, sY, G, ldg, sG, ncol, r0, mid, s));
  GemmDesc g{};
  g.M = r1 - mid; g.N = ncol; g.K = mid - r0;
  g.A = F.L + mid * F.ld + r0; g.lda = F.ld; g.at = 0;
  g.B = G + r0 * ldg; g.ldb = ldg; g.bt = 0;
  g.C = Y + mid * ldy; g.ldc = ldy;
  g.alpha = -1.0; g.beta = 1.0; g.lower = 0;
  g.batch = batch; g.sA = F.sL; g.sB = sG; g.sC = sY;
  g.mode = F.mode;
  CF_HIP_TRY(gemm_f64(g, s));
  return trsm_rec(F, Y, ldy, sY, G, ldg, sG, ncol, mid, r1, s);
}
}  // namespace

hipError_t trsm_lower_f64(const Factor& F, double* Y, int64_t ldy, int64_t sY, double* G, int64_t ldg,
                          int64_t sG, int64_t ncol, int64_t r0, hipStream_t s) {
  if (ncol <= 0 || F.n <= 0) return hipSuccess;
  const int64_t start = (r0 / NB) * NB;
  return trsm_rec(F, Y, ldy, sY, G, ldg, sG, ncol, start, F.n, s);
}

namespace {
// X[r0:r1] = L[r0:r1, r0:r1]^-T B[r0:r1] (B consumed).  Bottom half first, then
// B[r0:mid] -= L[mid:r1, r0:mid]^T X[mid:r1], then the top half; leaves use the transposed
// inverted diagonal blocks.
hipError_t trsmt_rec(const Factor& F, double* B, int64_t ldb, int64_t sB, double* X, int64_t ldx,
                     int64_t sX, int64_t ncol, int64_t r0, int64_t r1, hipStream_t s) {
  const int batch = F.batch > 0 ? F.batch : 1;
  const bool leaf256 = F.Li256 && (r0 % 256) == 0 && r1 - r0 == 256;
  if (r1 - r0 <= NB || leaf256) {
    const int64_t m = r1 - r0;
    GemmDesc g{};
    g.M = m; g.N = ncol; g.K = m;
    if (leaf256) { g.A = F.Li256 + (r0 / 256) * 256 * 256; g.lda = 256; g.sA = F.sLi256; }
    else { g.A = F.Li64 + (r0 / NB) * NB * NB; g.lda = NB; g.sA = F.sLi64; }
    g.at = 1;
    g.B = B + r0 * ldb; g.ldb = ldb; g.bt = 0;
    g.C = X + r0 * ldx; g.ldc = ldx;
    g.alpha = 1.0; g.beta = 0.0;
    g.batch = batch; g.sB = sB; g.sC = sX;
    g.mode = F.mode;
    return gemm_f64(g, s);
  }
  int64_t mid;
  const int64_t up = ((r0 + 255) / 256) * 256;
  if (F.Li256 && r0 % 256 != 0 && up < r1) {
    mid = up;
  } else if (F.Li256 && r0 % 256 == 0 && r1 - r0 > 256) {
    const int64_t n256 = (r1 - r0 + 255) / 256;
    mid = r0 + ((n256 + 1) / 2) * 256;
    if (mid >= r1) mid = r0 + 256;
  } else {
    const int64_t nblk = (r1 - r0 + NB - 1) / NB;
    mid = r0 + ((nblk + 1) / 2) * NB;
  }
  CF_HIP_TRY(trsmt_rec(F, B, ldb, sB, X, ldx, sX, ncol, mid, r1, s));
  GemmDesc g{};
  g.M = mid - r0; g.N = ncol; g.K = r1 - mid;
  g.A = F.L + mid * F.ld + r0; g.lda = F.ld; g.at = 1;     // A(i,k) = L[mid+k][r0+i]
  g.B = X + mid * ldx; g.ldb = ldx; g.bt = 0;
  g.C = B + r0 * ldb; g.ldc = ldb;
  g.alpha = -1.0; g.beta = 1.0;
  g.batch = batch; g.sA = F.sL; g.sB = sX; g.sC = sB;
  g.mode = F.mode;
  CF_HIP_TRY(gemm_f64(g, s));
  return trsmt_rec(F, B, ldb, sB, X, ldx, sX, ncol, r0, mid, s);
}
}  // namespace

hipError_t trsm_lower_t_f64(const Factor& F, double* B, int64_t ldb, int64_t sB, double* X, int64_t ldx,
                            int64_t sX, int64_t ncol, hipStream_t s) {
  if (ncol <= 0 || F.n <= 0) return hipSuccess;
  return trsmt_rec(F, B, ldb, sB, X, ldx, sX, ncol, 0, F.n, s);
}

}  // namespace cf
