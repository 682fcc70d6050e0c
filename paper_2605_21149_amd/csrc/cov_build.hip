// Pixel covariance assembly C = S + N (paper Eqs. total_cov, signal_cov; App. A spin-2 pieces).
//
// One thread per ordered pixel pair (i, j): the Legendre and spin-2 recurrences run in
// registers over l, accumulating the correlation sums
//   xi_TT = sum c^TT_l P_l,  xi_+ = sum (c^EE_l + c^BB_l) d^l_22,  xi_- = sum (c^EE_l - c^BB_l) d^l_2-2,
//   xi_EB = sum c^EB_l d^l_2-2,  xi_TE = sum c^TE_l d^l_20,  xi_TB = sum c^TB_l d^l_20,
// with c^XY_l = (2l+1)/(4 pi) C^XY_l W_l.  These are the correlations in the frame of the great
// circle through the pair; they are rotated to each pixel's local (theta, phi) frame with the
// angles psi_i, psi_j between the local meridians and that great circle (App. A.4):
//   <P_i P_j*> = e^{2i(psi_i - psi_j)} xi_+ ,  <P_i P_j> = e^{2i(psi_i + psi_j)} (xi_- + 2i xi_EB),
//   <T_i P_j*> = -e^{-2i psi_j} (xi_TE - i xi_TB),  <P_i T_j> = -e^{2i psi_i} (xi_TE + i xi_TB),
// with P = Q + iU.  cos 2psi, sin 2psi come from the tangent components (a, b) of the other
// pixel's direction without trigonometry; coincident and antipodal pairs take the meridian.
// Consecutive threads own consecutive j, so every store of the outputs is coalesced.
#include "cf_internal.h"

namespace cf {
namespace {

// IB points of a scan share one pixel pair: the recurrences (which depend only on the pair) run
// once and feed IB sets of sums, and the noise entry is read once for all of them.  IB == 1 reads
// weights laid out [item][field][l] (item stride cw_stride); IB > 1 reads the interleaved layout
// [chunk][l][field][IB] (chunk stride cw_stride), zero-padded past the last point, so that the
// 6 * IB weights of one l are contiguous.  Every point's sums follow the same operation order as
// with IB == 1, so results do not depend on how points are grouped.
template <int FIELDS, int IB>
__global__ __launch_bounds__(256) void k_cov_build(
    const double* __restrict__ pix, int npx, int n, int lmax, const double* __restrict__ coef,
    const double* __restrict__ cw_base, int64_t cw_stride, int nitems, int noise_kind,
    const double* __restrict__ noise, int noise_rank, const double* __restrict__ noise_U,
    double* __restrict__ C_base, int64_t ldc, int64_t c_stride, int lower_only, int* flag) {
  constexpr bool HT = (FIELDS & 1) != 0;   // T present
  constexpr bool HP = (FIELDS & 2) != 0;   // Q, U present
  constexpr int NM = (HT ? 1 : 0) + (HP ? 2 : 0);
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int item0 = blockIdx.z * IB;
  if (i >= npx || j >= npx) return;
  const int cnt = nitems - item0 < IB ? nitems - item0 : IB;
  const int L = lmax + 1;
  const double* cw = cw_base + (int64_t)blockIdx.z * cw_stride;
  auto W = [&](int x, int l, int t) -> double {
    return IB == 1 ? cw[x * L + l] : cw[((int64_t)l * 6 + x) * IB + t];
  };

  const double* pi = pix + (int64_t)i * kPixRec;
  const double* pj = pix + (int64_t)j * kPixRec;
  double mu = pi[0] * pj[0] + pi[1] * pj[1] + pi[2] * pj[2];
  mu = fmin(1.0, fmax(-1.0, mu));

  double xtt[IB], xp[IB], xm[IB], xeb[IB], xte[IB], xtb[IB];
#pragma unroll
  for (int t = 0; t < IB; ++t) xtt[t] = xp[t] = xm[t] = xeb[t] = xte[t] = xtb[t] = 0.0;
  if (HT) {
    double p0 = 1.0, p1 = mu;
#pragma unroll
    for (int t = 0; t < IB; ++t) xtt[t] = W(0, 0, t) + (lmax >= 1 ? W(0, 1, t) * mu : 0.0);
    for (int l = 1; l < lmax; ++l) {
      const double* q = coef + l * kCoef;
      double p2 = q[0] * mu * p1 - q[1] * p0;
#pragma unroll
      for (int t = 0; t < IB; ++t) xtt[t] = fma(W(0, l + 1, t), p2, xtt[t]);
      p0 = p1; p1 = p2;
    }
  }
  if (HP && lmax >= 2) {
    double hp = 0.5 * (1.0 + mu), hm = 0.5 * (1.0 - mu);
    double a0 = 0.0, a1 = hp * hp;          // d^l_22 at l-1, l
    double b0 = 0.0, b1 = hm * hm;          // d^l_2-2
    double c0 = 0.0, c1 = 0.6123724356957945 * (1.0 - mu * mu);   // d^l_20, sqrt(6)/4
    for (int l = 2;; ++l) {
#pragma unroll
      for (int t = 0; t < IB; ++t) {
        const double ee = W(1, l, t), bb = W(2, l, t);
        double sp = ee + bb, sm = ee - bb;
        xp[t] = fma(sp, a1, xp[t]);
        xm[t] = fma(sm, b1, xm[t]);
        xeb[t] = fma(W(5, l, t), b1, xeb[t]);
        if (HT) {
          xte[t] = fma(W(3, l, t), c1, xte[t]);
          xtb[t] = fma(W(4, l, t), c1, xtb[t]);
        }
      }
      if (l == lmax) break;
      const double* q = coef + l * kCoef;
      double tq = q[2] * mu;
      double a2 = (tq - q[3]) * a1 - q[4] * a0;
      double b2 = (tq + q[3]) * b1 - q[4] * b0;
      a0 = a1; a1 = a2; b0 = b1; b1 = b2;
      if (HT) {
        double c2 = q[5] * mu * c1 - q[6] * c0;
        c0 = c1; c1 = c2;
      }
    }
  }

  // rotation to the pixels' local frames (depends on the pair only)
  double rm = 0, im = 0, rp = 0, ip = 0, c2i = 0, s2i = 0, c2j = 0, s2j = 0;
  if (HP) {
    // psi_i: at pixel i toward j; psi_j: at pixel j toward i (tangent components of the other n)
    double ai = pj[0] * pi[3] + pj[1] * pi[4] + pj[2] * pi[5];
    double bi = pj[0] * pi[6] + pj[1] * pi[7];
    double aj = pi[0] * pj[3] + pi[1] * pj[4] + pi[2] * pj[5];
    double bj = pi[0] * pj[6] + pi[1] * pj[7];
    double ri = ai * ai + bi * bi, rj = aj * aj + bj * bj;
    if (ri < 1e-12) { ai = 1.0; bi = 0.0; ri = 1.0; }
    if (rj < 1e-12) { aj = 1.0; bj = 0.0; rj = 1.0; }
    c2i = (ai * ai - bi * bi) / ri; s2i = 2.0 * ai * bi / ri;
    c2j = (aj * aj - bj * bj) / rj; s2j = 2.0 * aj * bj / rj;
    rm = c2i * c2j + s2i * s2j; im = s2i * c2j - c2i * s2j;   // e^{2i(psi_i - psi_j)}
    rp = c2i * c2j - s2i * s2j; ip = s2i * c2j + c2i * s2j;   // e^{2i(psi_i + psi_j)}
  }
  // entry (a, b) of the NM x NM pixel-pair block for point t
  auto entry = [&](int a, int b, int t) -> double {
    const int k0 = HT ? 1 : 0;
    if (HT && a == 0 && b == 0) return xtt[t];
    if (HP && a >= k0 && b >= k0) {
      const double ppc_r = rm * xp[t], ppc_i = im * xp[t];
      const double pp_r = rp * xm[t] - 2.0 * ip * xeb[t], pp_i = ip * xm[t] + 2.0 * rp * xeb[t];
      if (a == k0 && b == k0) return 0.5 * (ppc_r + pp_r);           // Q_i Q_j
      if (a == k0 + 1 && b == k0 + 1) return 0.5 * (ppc_r - pp_r);   // U_i U_j
      if (a == k0) return 0.5 * (pp_i - ppc_i);                      // Q_i U_j
      return 0.5 * (pp_i + ppc_i);                                   // U_i Q_j
    }
    if (a == 0 && b == 1) return -(c2j * xte[t] - s2j * xtb[t]);     // T_i Q_j
    if (a == 0 && b == 2) return -(c2j * xtb[t] + s2j * xte[t]);     // T_i U_j
    if (a == 1 && b == 0) return -(c2i * xte[t] - s2i * xtb[t]);     // Q_i T_j
    return -(s2i * xte[t] + c2i * xtb[t]);                           // U_i T_j
  };

#pragma unroll
  for (int a = 0; a < NM; ++a) {
#pragma unroll
    for (int b = 0; b < NM; ++b) {
      const int64_t row = (int64_t)a * npx + i;
      const int64_t col = (int64_t)b * npx + j;
      if (lower_only && col > row) continue;
      double nv = 0.0;
      const bool add_n = noise_kind == 1 || row == col;
      if (noise_kind == 1) nv = noise[row * n + col];
      else if (row == col) nv = noise[row];
#pragma unroll
      for (int t = 0; t < IB; ++t) {
        if (t >= cnt) break;
        double v = entry(a, b, t);
        if (add_n) v += nv;
        for (int r = 0; r < noise_rank; ++r)
          v = fma(noise_U[row * noise_rank + r], noise_U[col * noise_rank + r], v);
        if (!isfinite(v)) atomicOr(flag, 1);
        C_base[(int64_t)(item0 + t) * c_stride + row * ldc + col] = v;
      }
    }
  }
}

}  // namespace

hipError_t launch_cov_build(const DevProblem& P, const double* cw, int64_t cw_stride, int nbatch,
                            int noise_kind, const double* noise, int noise_rank,
                            const double* noise_U, double* C, int64_t ldc, int64_t c_stride,
                            int lower_only, int* flag, hipStream_t s, int interleave) {
  if (P.npx <= 0 || nbatch <= 0) return hipSuccess;
  if (interleave != 1 && interleave != kCovIB) return hipErrorInvalidValue;
  const int chunks = (nbatch + interleave - 1) / interleave;
  dim3 grid((P.npx + 63) / 64, (P.npx + 3) / 4, chunks), block(256);
  int fields = (P.has_t ? 1 : 0) | (P.has_p ? 2 : 0);
#define CF_COV_ARGS P.pix, P.npx, P.n, P.lmax, P.coef, cw, cw_stride, nbatch, noise_kind, noise, \
                    noise_rank, noise_U, C, ldc, c_stride, lower_only, flag
#define CF_COV_CASE(F)                                                                          \
  if (interleave == 1) hipLaunchKernelGGL((k_cov_build<F, 1>), grid, block, 0, s, CF_COV_ARGS); \
  else hipLaunchKernelGGL((k_cov_build<F, kCovIB>), grid, block, 0, s, CF_COV_ARGS);
  switch (fields) {
    case 1: CF_COV_CASE(1) break;
    case 2: CF_COV_CASE(2) break;
    case 3: CF_COV_CASE(3) break;
    default: return hipErrorInvalidValue;
  }
#undef CF_COV_CASE
#undef CF_COV_ARGS
  return hipGetLastError();
}

}  // namespace cf
