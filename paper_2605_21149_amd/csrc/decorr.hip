// Decorrelated normalisation (Sect. 2.5, Eq. decorrelated): C^decorr = F^-1/2 q with
// F^-1/2 = U Xi^-1/2 U^T from the eigendecomposition F = U Xi U^T, eigenvalues below 1e-12 of the
// largest set to zero.
//
// The eigendecomposition is a cyclic Jacobi iteration in one workgroup.  A sweep is K' - 1 rounds
// of the round-robin schedule over K' = K rounded up to even indices; a round rotates K'/2
// disjoint index pairs at once: the rotation of every pair is computed from the matrix as it
// stands before the round (the 2 x 2 symmetric Schur decomposition that zeroes a_pq), then all
// pairs' rows of A are rotated, then all pairs' columns of A and of U.  A pair is left alone when
// |a_pq| <= max(1e-15 sqrt(|a_pp a_qq|), 2e-17 |A|_F): the relative threshold keeps the small
// eigenvalues accurate whatever the conditioning, the absolute floor (below the matrix's rounding
// level) lets a singular matrix's null space settle.  The iteration stops after a sweep without
// rotations, or after max_sweeps.
#include "cf_internal.h"

namespace cf {
namespace {

constexpr int kJT = 1024;   // threads of the Jacobi workgroup; K <= 2 * 512 pairs

__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

// A: [K][K] symmetric (overwritten: its diagonal ends as the eigenvalues), U: [K][K] eigenvectors
// as columns, w: [K] weights Xi^-1/2 after the cutoff, info[0]: sweeps run, info[1]: 1 when the
// tolerance was not reached.
__global__ __launch_bounds__(kJT) void k_jacobi(double* __restrict__ A, double* __restrict__ U,
                                                double* __restrict__ w, int K, int max_sweeps,
                                                double cutoff, int* info) {
  __shared__ double cs[kJT / 2], sn[kJT / 2];
  __shared__ int pp[kJT / 2], qq[kJT / 2];
  __shared__ double red[kJT / 64];
  __shared__ int nrot;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int Kp = K + (K & 1), np = Kp / 2;
  double nrm = 0.0;
  for (int i = tid; i < K * K; i += nt) {
    U[i] = (i / K == i % K) ? 1.0 : 0.0;
    nrm += A[i] * A[i];
  }
  // rounding level of the whole matrix: off-diagonal entries below it count as zero (without this
  // floor the null space of a singular F keeps receiving rotation noise from its other rows)
  const double floor_abs = 2e-17 * sqrt(block_sum(nrm, red));
  int sweep = 0;
  bool converged = false;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) nrot = 0;
    __syncthreads();
    for (int r = 0; r < Kp - 1; ++r) {
      for (int k = tid; k < np; k += nt) {
        int a, b;
        if (k == 0) { a = r; b = Kp - 1; }
        else { a = (r + k) % (Kp - 1); b = (r - k + (Kp - 1)) % (Kp - 1); }
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (q < K) {
          const double apq = A[p * K + q], app = A[p * K + p], aqq = A[q * K + q];
          if (fabs(apq) > fmax(1e-15 * sqrt(fabs(app * aqq)), floor_abs) && apq != 0.0) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            nrot = 1;
          }
        }
        pp[k] = p; qq[k] = q; cs[k] = c; sn[k] = s;
      }
      __syncthreads();
      for (int idx = tid; idx < np * K; idx += nt) {       // rows p, q of A <- J^T A
        const int k = idx / K, j = idx % K, p = pp[k], q = qq[k];
        if (q >= K) continue;
        const double c = cs[k], s = sn[k], x = A[p * K + j], y = A[q * K + j];
        A[p * K + j] = c * x - s * y;
        A[q * K + j] = s * x + c * y;
      }
      __syncthreads();
      for (int idx = tid; idx < np * K; idx += nt) {       // columns p, q of A <- A J, U <- U J
        const int k = idx / K, i = idx % K, p = pp[k], q = qq[k];
        if (q >= K) continue;
        const double c = cs[k], s = sn[k];
        double x = A[i * K + p], y = A[i * K + q];
        A[i * K + p] = c * x - s * y;
        A[i * K + q] = s * x + c * y;
        x = U[i * K + p]; y = U[i * K + q];
        U[i * K + p] = c * x - s * y;
        U[i * K + q] = s * x + c * y;
      }
      __syncthreads();
    }
    if (nrot == 0) { converged = true; break; }   // read after the round's last barrier
    __syncthreads();                               // before the next sweep resets nrot
  }
  // weights Xi^-1/2 with the cutoff relative to the largest eigenvalue
  double mx = -INFINITY;
  for (int i = tid; i < K; i += nt) mx = fmax(mx, A[i * K + i]);
  {
    const int lane = tid & 63, wave = tid >> 6;
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    mx = -INFINITY;
    for (int v = 0; v < nt / 64; ++v) mx = fmax(mx, red[v]);
  }
  for (int i = tid; i < K; i += nt) {
    const double xi = A[i * K + i];
    w[i] = (mx > 0.0 && xi > cutoff * mx) ? 1.0 / sqrt(xi) : 0.0;
  }
  if (tid == 0) {
    info[0] = sweep;
    info[1] = converged ? 0 : 1;
  }
}

// A <- F with the upper triangle mirrored from the lower one.
__global__ void k_sym_from_lower(const double* __restrict__ F, double* __restrict__ A, int K) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)K * K) return;
  const int i = (int)(idx / K), j = (int)(idx % K);
  A[idx] = j <= i ? F[(int64_t)i * K + j] : F[(int64_t)j * K + i];
}

// R = U diag(w) U^T
__global__ void k_inv_sqrt_form(const double* __restrict__ U, const double* __restrict__ w, int K,
                                double* __restrict__ R) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)K * K) return;
  const int i = (int)(idx / K), j = (int)(idx % K);
  double s = 0.0;
  for (int k = 0; k < K; ++k) s = fma(U[(int64_t)i * K + k] * w[k], U[(int64_t)j * K + k], s);
  R[idx] = s;
}

// out[v][i] = sum_j R[i][j] q[v][j]
__global__ void k_apply_rows(const double* __restrict__ R, const double* __restrict__ q, int K, int nvec,
                             double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)K * nvec) return;
  const int v = (int)(idx / K), i = (int)(idx % K);
  double s = 0.0;
  for (int j = 0; j < K; ++j) s = fma(R[(int64_t)i * K + j], q[(int64_t)v * K + j], s);
  out[idx] = s;
}

}  // namespace

hipError_t launch_inverse_sqrt(const double* F, int K, double* A, double* U, double* w, double* R,
                               int max_sweeps, double cutoff, int* info, hipStream_t s) {
  if (K <= 0 || K > kJT) return hipErrorInvalidValue;
  const int64_t kk = (int64_t)K * K;
  hipLaunchKernelGGL(k_sym_from_lower, dim3((unsigned)((kk + 255) / 256)), dim3(256), 0, s, F, A, K);
  CF_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kJT), 0, s, A, U, w, K, max_sweeps, cutoff, info);
  CF_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_inv_sqrt_form, dim3((unsigned)((kk + 255) / 256)), dim3(256), 0, s, U, w, K, R);
  return hipGetLastError();
}

hipError_t launch_apply_rows(const double* R, const double* q, int K, int nvec, double* out, hipStream_t s) {
  const int64_t n = (int64_t)K * nvec;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_apply_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, R, q, K, nvec, out);
  return hipGetLastError();
}

}  // namespace cf
