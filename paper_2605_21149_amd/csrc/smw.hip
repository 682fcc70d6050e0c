// Pixel likelihood through the harmonic basis with multipole switching: the per-point kernels
// (Sects. 2.3.2, 2.3.4, 2.6; Eqs. C_switched, N_eff, K_kernel, smw, logdet; App. smw_stable).
//
// The window's modes are ordered [field][l][m] over the varied fields (the order of Y's columns),
// so mode i of a window of kwf modes per field is field slot i / kwf at r = i % kwf, with
// l = floor(sqrt(r + wlo^2)).  With Lambda_l = R_l R_l^T over the varied fields and
// M = V N_eff^-1 V^T, b = V N_eff^-1 d, the per-point system is
//   K' = I + R^T M R,   b' = R^T b,
//   d^T C^-1 d = d^T N_eff^-1 d - |L_K'^-1 b'|^2,   ln|C| = ln|N_eff| + ln|K'|,
// which is Eq. smw with Eq. logdet after K = Lambda^-1 + M = R^-T K' R^-1.  K' has eigenvalues
// >= 1 at any signal-to-noise ratio (the argument of App. smw_stable), needs no inverse of
// Lambda, and a field without power at some l simply contributes a zero column of R.
#include "cf_internal.h"

#include <algorithm>

namespace cf {
namespace {

// spectrum row (TT, EE, BB, TE, TB, EB) of the harmonic field pair (a, b), fields T 0, E 1, B 2
__device__ __forceinline__ int spec_of(int a, int b) {
  if (a > b) { const int t = a; a = b; b = t; }
  if (a == b) return a;
  if (a == 0) return b == 1 ? 3 : 4;
  return 5;
}

__device__ __forceinline__ int ell_of(int64_t r, int wlo) {
  const int64_t w2 = (int64_t)wlo * wlo;
  int l = (int)sqrt((double)(r + w2));
  while ((int64_t)(l + 1) * (l + 1) - w2 <= r) ++l;
  while ((int64_t)l * l - w2 > r) --l;
  return l;
}

// R_l for every point of the batch and every l of the window: the lower Cholesky factor of
// Lambda_l = [C^{f_a f_b}_l W_l] over the varied fields, a zero pivot giving a zero column.
// bad: smallest l whose Lambda_l is not positive semi-definite (or not finite).
__global__ void k_smw_lambda(const double* __restrict__ cl, int64_t cl_stride, int64_t cl_ld,
                             const double* __restrict__ wl, int wlo, int nl, int nf, int f0, int f1,
                             int f2, double* __restrict__ R, int* bad) {
  const int lo = blockIdx.x * blockDim.x + threadIdx.x;
  const int pt = blockIdx.y;
  if (lo >= nl) return;
  const int l = wlo + lo;
  const int fld[3] = {f0, f1, f2};
  const double* c = cl + (int64_t)pt * cl_stride;
  const double W = wl[l];
  double A[3][3], Lr[3][3];
  double scale = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      A[a][b] = (a < nf && b < nf) ? c[(int64_t)spec_of(fld[a], fld[b]) * cl_ld + l] * W : 0.0;
      Lr[a][b] = 0.0;
    }
  for (int a = 0; a < nf; ++a) scale = fmax(scale, fabs(A[a][a]));
  bool ok = isfinite(scale);
  for (int j = 0; j < nf; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= Lr[j][k] * Lr[j][k];
    if (d > 1e-13 * scale) {
      const double r = sqrt(d);
      Lr[j][j] = r;
      for (int i = j + 1; i < nf; ++i) {
        double t = A[i][j];
        for (int k = 0; k < j; ++k) t -= Lr[i][k] * Lr[j][k];
        Lr[i][j] = t / r;
      }
    } else {
      // semi-definite: the rest of the column must vanish as well
      if (d < -1e-10 * scale) ok = false;
      for (int i = j + 1; i < nf; ++i) {
        double t = A[i][j];
        for (int k = 0; k < j; ++k) t -= Lr[i][k] * Lr[j][k];
        if (fabs(t) > 1e-10 * scale) ok = false;
      }
    }
  }
  if (!ok) atomicMin(bad, l);
  double* out = R + ((int64_t)pt * nl + lo) * 9;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) out[a * 3 + b] = Lr[a][b];
}

// K' = I + R^T M R for every point: one thread per (r_i, r_j) reads the nf x nf field block of M
// at those positions once and writes the lower-triangle entries of K' for all field pairs.
// M: [kw][kw] (leading dimension ldm: a diagonal block of a larger M for one field group),
// K': slot of [kw + nmaps][kw] per point (the first kw rows).
__global__ __launch_bounds__(256) void k_smw_kernel(const double* __restrict__ M, int64_t ldm, int64_t kw,
                                                    int64_t kwf, int nf, int wlo, int nl,
                                                    const double* __restrict__ R, double* __restrict__ K,
                                                    int64_t slot) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int pt = blockIdx.y;
  if (t >= kwf * kwf) return;
  const int64_t ri = t / kwf, rj = t % kwf;
  const double* Ri = R + ((int64_t)pt * nl + (ell_of(ri, wlo) - wlo)) * 9;
  const double* Rj = R + ((int64_t)pt * nl + (ell_of(rj, wlo) - wlo)) * 9;
  double Mv[3][3];
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) Mv[c][d] = (c < nf && d < nf) ? M[(c * kwf + ri) * ldm + d * kwf + rj] : 0.0;
  double* Kp = K + (int64_t)pt * slot;
  for (int fi = 0; fi < nf; ++fi)
    for (int fj = 0; fj < nf; ++fj) {
      double v = 0.0;
      for (int c = fi; c < nf; ++c) {
        double s = 0.0;
        for (int d = fj; d < nf; ++d) s = fma(Mv[c][d], Rj[d * 3 + fj], s);
        v = fma(Ri[c * 3 + fi], s, v);
      }
      if (fi == fj && ri == rj) v += 1.0;
      const int64_t row = fi * kwf + ri, col = fj * kwf + rj;
      if (col <= row) Kp[row * kw + col] = v;   // the factorisation reads the lower triangle only
    }
}

// b' = R^T b into the rows below K' (row kw + j holds map j): b [kw][nmaps].
__global__ void k_smw_rhs(const double* __restrict__ b, int nmaps, int64_t kw, int64_t kwf, int nf,
                          int wlo, int nl, const double* __restrict__ R, double* __restrict__ K,
                          int64_t slot) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int pt = blockIdx.y;
  if (t >= kw * nmaps) return;
  const int64_t j = t / kw, i = t % kw;
  const int fi = (int)(i / kwf);
  const int64_t ri = i % kwf;
  const double* Ri = R + ((int64_t)pt * nl + (ell_of(ri, wlo) - wlo)) * 9;
  double v = 0.0;
  for (int c = fi; c < nf; ++c) v = fma(Ri[c * 3 + fi], b[(c * kwf + ri) * nmaps + j], v);
  K[(int64_t)pt * slot + (kw + j) * kw + i] = v;
}

// flag[0] = 1 if any entry of a rows x cols block (leading dimension ld, batch stride sb over nb
// items) is non-zero or not finite: the coupling block of M between field groups, or the coupling
// spectra of the points inside the window.
__global__ void k_any_nonzero(const double* __restrict__ A, int64_t ld, int64_t rows, int64_t cols, int64_t sb,
                              int nb, int* flag) {
  const int64_t total = rows * cols * nb;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = t / (rows * cols), r = (t / cols) % rows, c = t % cols;
    if (A[z * sb + r * ld + c] != 0.0) {   // also true for NaN
      atomicOr(flag, 1);
      return;
    }
  }
}

// The per-mode block operator B built from R (one point): B[(f,r),(g,r')] = delta_rr' X_l(r)[f][g]
// with X = R (kind 0), R^T (1), R^-1 (2) or R^-T (3) over the nf window fields; applied on the
// left (out = B A) or on the right (out = A B) of a k x ncol (left) or nrow x k (right) matrix.
__device__ __forceinline__ void rblock(const double* Rl, int kind, double X[3][3]) {
  double Li[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  if (kind >= 2) {                       // inverse of the lower factor, column by column
    for (int j = 0; j < 3; ++j) {
      const double d = Rl[j * 3 + j];
      Li[j][j] = d != 0.0 ? 1.0 / d : 0.0;
      for (int i = j + 1; i < 3; ++i) {
        double t = 0.0;
        for (int q = j; q < i; ++q) t += Rl[i * 3 + q] * Li[q][j];
        Li[i][j] = Rl[i * 3 + i] != 0.0 ? -t / Rl[i * 3 + i] : 0.0;
      }
    }
  }
  for (int f = 0; f < 3; ++f)
    for (int g = 0; g < 3; ++g) {
      const double r = kind == 0 ? Rl[f * 3 + g] : kind == 1 ? Rl[g * 3 + f] : kind == 2 ? Li[f][g] : Li[g][f];
      X[f][g] = r;
    }
}

__global__ void k_apply_rblock(const double* __restrict__ A, int64_t lda, double* __restrict__ out, int64_t ldo,
                               int64_t other, int64_t kwf, int nf, int wlo, const double* __restrict__ R, int kind,
                               int right) {
  const int64_t kw = kwf * nf;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kw * other) return;
  // the mode index of the output entry and its index along the other dimension (the fastest
  // running one is the contiguous one of the output)
  const int64_t mode = right ? t % kw : t / other;
  const int64_t oth = right ? t / kw : t % other;
  const int f = (int)(mode / kwf);
  const int64_t r = mode % kwf;
  double X[3][3];
  rblock(R + (int64_t)(ell_of(r, wlo) - wlo) * 9, kind, X);
  double v = 0.0;
  if (right) {                          // out[oth][(f, r)] = sum_c A[oth][(c, r)] X[c][f]
    for (int c = 0; c < nf; ++c) v = fma(A[oth * lda + c * kwf + r], X[c][f], v);
    out[oth * ldo + mode] = v;
  } else {                              // out[(f, r)][oth] = sum_c X[f][c] A[(c, r)][oth]
    for (int c = 0; c < nf; ++c) v = fma(X[f][c], A[(c * kwf + r) * lda + oth], v);
    out[mode * ldo + oth] = v;
  }
}

// -2 ln L = d^T N_eff^-1 d - |L^-1 b'|^2 + ln|N_eff| + ln|K'| for the points of one batch.
__global__ void k_smw_finish(const double* chi2N, const double* ldN, const double* x2b, const double* ldK,
                             int B, int nmaps, int64_t i0, double* m2, double* chi2, double* logdet) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * nmaps) return;
  const int b = idx / nmaps, j = idx % nmaps;
  const double x = chi2N[j] - x2b[idx], l = ldN[0] + ldK[b];
  const int64_t row = i0 + b;
  m2[row * nmaps + j] = x + l;
  if (chi2) chi2[row * nmaps + j] = x;
  if (logdet && j == 0) logdet[row] = l;
}

}  // namespace

hipError_t launch_smw_lambda(const double* cl, int64_t cl_stride, int64_t cl_ld, const double* wl, int wlo,
                             int nl, int nf, const int* fld, int batch, double* R, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_smw_lambda, dim3((nl + 63) / 64, batch), dim3(64), 0, s, cl, cl_stride, cl_ld, wl,
                     wlo, nl, nf, fld[0], fld[1], fld[2], R, bad);
  return hipGetLastError();
}

hipError_t launch_smw_kernel(const double* M, int64_t ldm, int64_t kw, int64_t kwf, int nf, int wlo, int nl,
                             const double* R, int batch, double* K, int64_t slot, hipStream_t s) {
  const int64_t nt = kwf * kwf;
  hipLaunchKernelGGL(k_smw_kernel, dim3((unsigned)((nt + 255) / 256), batch), dim3(256), 0, s, M, ldm, kw, kwf,
                     nf, wlo, nl, R, K, slot);
  return hipGetLastError();
}

hipError_t launch_apply_rblock(const double* A, int64_t lda, double* out, int64_t ldo, int64_t other, int64_t kwf,
                              int nf, int wlo, const double* R, int kind, int right, hipStream_t s) {
  const int64_t total = kwf * nf * other;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_apply_rblock, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, A, lda, out, ldo, other,
                     kwf, nf, wlo, R, kind, right);
  return hipGetLastError();
}

hipError_t launch_any_nonzero(const double* A, int64_t ld, int64_t rows, int64_t cols, int64_t sb, int nb,
                              int* flag, hipStream_t s) {
  if (rows <= 0 || cols <= 0 || nb <= 0) return hipSuccess;
  const int64_t total = rows * cols * nb;
  const unsigned blocks = (unsigned)std::min<int64_t>(2048, (total + 255) / 256);
  hipLaunchKernelGGL(k_any_nonzero, dim3(blocks), dim3(256), 0, s, A, ld, rows, cols, sb, nb, flag);
  return hipGetLastError();
}

hipError_t launch_smw_rhs(const double* b, int nmaps, int64_t kw, int64_t kwf, int nf, int wlo, int nl,
                          const double* R, int batch, double* K, int64_t slot, hipStream_t s) {
  const int64_t nt = kw * nmaps;
  hipLaunchKernelGGL(k_smw_rhs, dim3((unsigned)((nt + 255) / 256), batch), dim3(256), 0, s, b, nmaps, kw, kwf,
                     nf, wlo, nl, R, K, slot);
  return hipGetLastError();
}

hipError_t launch_smw_finish(const double* chi2N, const double* ldN, const double* x2b, const double* ldK,
                             int B, int nmaps, int64_t i0, double* m2, double* chi2, double* logdet,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_smw_finish, dim3((B * nmaps + 255) / 256), dim3(256), 0, s, chi2N, ldN, x2b, ldK, B,
                     nmaps, i0, m2, chi2, logdet);
  return hipGetLastError();
}

}  // namespace cf
