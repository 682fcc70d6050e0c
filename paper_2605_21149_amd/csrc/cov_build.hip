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
// Consecutive threads own consecutive j, so every store of the nmaps^2 outputs is coalesced.
#include "cf_internal.h"

namespace cf {
namespace {

template <int FIELDS>
__global__ __launch_bounds__(256) void k_cov_build(
    const double* __restrict__ pix, int npx, int n, int lmax, const double* __restrict__ coef,
    const double* __restrict__ cw_base, int64_t cw_stride, int noise_kind,
    const double* __restrict__ noise, int noise_rank, const double* __restrict__ noise_U,
    double* __restrict__ C_base, int64_t ldc, int64_t c_stride, int lower_only, int* flag) {
  constexpr bool HT = (FIELDS & 1) != 0;   // T present
  constexpr bool HP = (FIELDS & 2) != 0;   // Q, U present
  constexpr int NM = (HT ? 1 : 0) + (HP ? 2 : 0);
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int item = blockIdx.z;
  if (i >= npx || j >= npx) return;
  const int L = lmax + 1;
  const double* cw = cw_base + (int64_t)item * cw_stride;
  double* C = C_base + (int64_t)item * c_stride;

  const double* pi = pix + (int64_t)i * kPixRec;
  const double* pj = pix + (int64_t)j * kPixRec;
  double mu = pi[0] * pj[0] + pi[1] * pj[1] + pi[2] * pj[2];
  mu = fmin(1.0, fmax(-1.0, mu));

  double xtt = 0, xp = 0, xm = 0, xeb = 0, xte = 0, xtb = 0;
  if (HT) {
    const double* ctt = cw;                         // TT row
    double p0 = 1.0, p1 = mu;
    xtt = ctt[0] + (lmax >= 1 ? ctt[1] * mu : 0.0);
    for (int l = 1; l < lmax; ++l) {
      const double* q = coef + l * kCoef;
      double p2 = q[0] * mu * p1 - q[1] * p0;
      xtt = fma(ctt[l + 1], p2, xtt);
      p0 = p1; p1 = p2;
    }
  }
  if (HP && lmax >= 2) {
    const double* cee = cw + 1 * L;
    const double* cbb = cw + 2 * L;
    const double* cte = cw + 3 * L;
    const double* ctb = cw + 4 * L;
    const double* ceb = cw + 5 * L;
    double hp = 0.5 * (1.0 + mu), hm = 0.5 * (1.0 - mu);
    double a0 = 0.0, a1 = hp * hp;          // d^l_22 at l-1, l
    double b0 = 0.0, b1 = hm * hm;          // d^l_2-2
    double c0 = 0.0, c1 = 0.6123724356957945 * (1.0 - mu * mu);   // d^l_20, sqrt(6)/4
    for (int l = 2;; ++l) {
      double sp = cee[l] + cbb[l], sm = cee[l] - cbb[l];
      xp = fma(sp, a1, xp);
      xm = fma(sm, b1, xm);
      xeb = fma(ceb[l], b1, xeb);
      if (HT) {
        xte = fma(cte[l], c1, xte);
        xtb = fma(ctb[l], c1, xtb);
      }
      if (l == lmax) break;
      const double* q = coef + l * kCoef;
      double t = q[2] * mu;
      double a2 = (t - q[3]) * a1 - q[4] * a0;
      double b2 = (t + q[3]) * b1 - q[4] * b0;
      a0 = a1; a1 = a2; b0 = b1; b1 = b2;
      if (HT) {
        double c2 = q[5] * mu * c1 - q[6] * c0;
        c0 = c1; c1 = c2;
      }
    }
  }

  double out[NM][NM];
  int k0 = 0;
  if (HT) { out[0][0] = xtt; k0 = 1; }
  if (HP) {
    // psi_i: at pixel i toward j; psi_j: at pixel j toward i (tangent components of the other n)
    double ai = pj[0] * pi[3] + pj[1] * pi[4] + pj[2] * pi[5];
    double bi = pj[0] * pi[6] + pj[1] * pi[7];
    double aj = pi[0] * pj[3] + pi[1] * pj[4] + pi[2] * pj[5];
    double bj = pi[0] * pj[6] + pi[1] * pj[7];
    double ri = ai * ai + bi * bi, rj = aj * aj + bj * bj;
    if (ri < 1e-12) { ai = 1.0; bi = 0.0; ri = 1.0; }
    if (rj < 1e-12) { aj = 1.0; bj = 0.0; rj = 1.0; }
    double c2i = (ai * ai - bi * bi) / ri, s2i = 2.0 * ai * bi / ri;
    double c2j = (aj * aj - bj * bj) / rj, s2j = 2.0 * aj * bj / rj;
    double rm = c2i * c2j + s2i * s2j, im = s2i * c2j - c2i * s2j;   // e^{2i(psi_i - psi_j)}
    double rp = c2i * c2j - s2i * s2j, ip = s2i * c2j + c2i * s2j;   // e^{2i(psi_i + psi_j)}
    double ppc_r = rm * xp, ppc_i = im * xp;
    double pp_r = rp * xm - 2.0 * ip * xeb, pp_i = ip * xm + 2.0 * rp * xeb;
    out[k0][k0] = 0.5 * (ppc_r + pp_r);             // Q_i Q_j
    out[k0 + 1][k0 + 1] = 0.5 * (ppc_r - pp_r);     // U_i U_j
    out[k0][k0 + 1] = 0.5 * (pp_i - ppc_i);         // Q_i U_j
    out[k0 + 1][k0] = 0.5 * (pp_i + ppc_i);         // U_i Q_j
    if (HT) {
      out[0][1] = -(c2j * xte - s2j * xtb);         // T_i Q_j
      out[0][2] = -(c2j * xtb + s2j * xte);         // T_i U_j
      out[1][0] = -(c2i * xte - s2i * xtb);         // Q_i T_j
      out[2][0] = -(s2i * xte + c2i * xtb);         // U_i T_j
    }
  }

#pragma unroll
  for (int a = 0; a < NM; ++a) {
#pragma unroll
    for (int b = 0; b < NM; ++b) {
      int64_t row = (int64_t)a * npx + i;
      int64_t col = (int64_t)b * npx + j;
      if (lower_only && col > row) continue;
      double v = out[a][b];
      if (noise_kind == 1) {
        v += noise[row * n + col];
      } else if (row == col) {
        v += noise[row];
      }
      for (int r = 0; r < noise_rank; ++r) v = fma(noise_U[row * noise_rank + r], noise_U[col * noise_rank + r], v);
      if (!isfinite(v)) atomicOr(flag, 1);
      C[row * ldc + col] = v;
    }
  }
}

}  // namespace

hipError_t launch_cov_build(const DevProblem& P, const double* cw, int64_t cw_stride, int nbatch,
                            int noise_kind, const double* noise, int noise_rank,
                            const double* noise_U, double* C, int64_t ldc, int64_t c_stride,
                            int lower_only, int* flag, hipStream_t s) {
  if (P.npx <= 0 || nbatch <= 0) return hipSuccess;
  dim3 grid((P.npx + 63) / 64, (P.npx + 3) / 4, nbatch), block(256);
  int fields = (P.has_t ? 1 : 0) | (P.has_p ? 2 : 0);
#define CF_COV_ARGS P.pix, P.npx, P.n, P.lmax, P.coef, cw, cw_stride, noise_kind, noise, noise_rank, \
                    noise_U, C, ldc, c_stride, lower_only, flag
  switch (fields) {
    case 1: hipLaunchKernelGGL(k_cov_build<1>, grid, block, 0, s, CF_COV_ARGS); break;
    case 2: hipLaunchKernelGGL(k_cov_build<2>, grid, block, 0, s, CF_COV_ARGS); break;
    case 3: hipLaunchKernelGGL(k_cov_build<3>, grid, block, 0, s, CF_COV_ARGS); break;
    default: return hipErrorInvalidValue;
  }
#undef CF_COV_ARGS
  return hipGetLastError();
}

}  // namespace cf
