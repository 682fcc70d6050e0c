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
// C is symmetric, so each unordered pair (i >= j) is computed once: a workgroup owns a 16 x 16
// tile of pairs from the lower triangle of tiles and writes each NM x NM block at (i, j) and,
// staged through LDS so that consecutive lanes again store consecutive columns, at (j, i).
// Dense noise is read at the position written (it may be a non-symmetric off-diagonal block).
#include "cf_internal.h"

namespace cf {
namespace {

// IB points of a scan share one pixel pair: the recurrences (which depend only on the pair) run
// once and feed IB sets of sums, and the noise entry is read once for all of them.  IB == 1 reads
// weights laid out [item][field][l] (item stride cw_stride); IB > 1 reads the interleaved layout
// [chunk][l][field][IB] (chunk stride cw_stride), zero-padded past the last point, so that the
// 6 * IB weights of one l are contiguous.  Every point's sums follow the same operation order as
// with IB == 1, so results do not depend on how points are grouped.
constexpr int kPT = 16;   // pixel-pair tile

template <int FIELDS, int IB>
__global__ __launch_bounds__(256) void k_cov_build(
    const double* __restrict__ pix, int npx, int n, int lmax, const double* __restrict__ coef,
    const double* __restrict__ cw_base, int64_t cw_stride, int nitems, int noise_kind,
    const double* __restrict__ noise, int noise_rank, const double* __restrict__ noise_U,
    double* __restrict__ C_base, int64_t ldc, int64_t c_stride, int lower_only, int* flag) {
  constexpr bool HT = (FIELDS & 1) != 0;   // T present
  constexpr bool HP = (FIELDS & 2) != 0;   // Q, U present
  constexpr int NM = (HT ? 1 : 0) + (HP ? 2 : 0);
  __shared__ double stage[IB][kPT][kPT + 1];   // signal entries for the mirrored stores
  __shared__ double stu[kPT][kPT + 1];          // and their U U^T terms
  // tile (I, J), I >= J, from the linear index k = I (I + 1) / 2 + J
  const int k = blockIdx.x;
  int I = (int)((sqrt(8.0 * k + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= k) ++I;
  while (I * (I + 1) / 2 > k) --I;
  const int J = k - I * (I + 1) / 2;
  const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
  const int i = I * kPT + ti, j = J * kPT + tj;
  // this thread's pair (i >= j); the others only take part in the staged stores
  const bool live = i < npx && j < npx && (I > J || ti >= tj);
  const int item0 = blockIdx.z * IB;
  const int cnt = nitems - item0 < IB ? nitems - item0 : IB;
  const int L = lmax + 1;
  const double* cw = cw_base + (int64_t)blockIdx.z * cw_stride;
  auto W = [&](int x, int l, int t) -> double {
    return IB == 1 ? cw[x * L + l] : cw[((int64_t)l * 6 + x) * IB + t];
  };

  // source pair of the value this thread stores at the mirrored position: (i, j) of thread (tj, ti)
  const int si = I * kPT + tj, sj = J * kPT + ti;
  const bool mlive = si < npx && sj < npx && (I > J || tj > ti);
  // noise entries at every position this thread stores, loaded before the recurrences so that
  // their latency (the dense matrix is read once, from HBM) hides behind them
  double nvd[NM][NM], nvm[NM][NM];
#pragma unroll
  for (int a = 0; a < NM; ++a)
#pragma unroll
    for (int b = 0; b < NM; ++b) {
      const int64_t row = (int64_t)a * npx + i, col = (int64_t)b * npx + j;
      nvd[a][b] = 0.0;
      if (live && !(lower_only && col > row)) {
        if (noise_kind == 1) nvd[a][b] = noise[row * n + col];
        else if (row == col) nvd[a][b] = noise[row];
      }
      const int64_t mrow = (int64_t)b * npx + sj, mcol = (int64_t)a * npx + si;
      nvm[a][b] = (mlive && noise_kind == 1 && !(lower_only && b <= a)) ? noise[mrow * n + mcol] : 0.0;
    }
  const double* pi = pix + (int64_t)(live ? i : 0) * kPixRec;
  const double* pj = pix + (int64_t)(live ? j : 0) * kPixRec;
  double mu = pi[0] * pj[0] + pi[1] * pj[1] + pi[2] * pj[2];
  mu = fmin(1.0, fmax(-1.0, mu));

  double xtt[IB], xp[IB], xm[IB], xeb[IB], xte[IB], xtb[IB];
#pragma unroll
  for (int t = 0; t < IB; ++t) xtt[t] = xp[t] = xm[t] = xeb[t] = xte[t] = xtb[t] = 0.0;
  // l = 0, 1 (temperature only), then one loop over l >= 2 carrying the Legendre recurrence and
  // the spin-2 ones.  The weights of the polarisation sums come as c^EE + c^BB and c^EE - c^BB.
  double pa = 1.0, pb = mu;                 // P_(l-1), P_l
  if (HT) {
#pragma unroll
    for (int t = 0; t < IB; ++t) xtt[t] = W(0, 0, t) + (lmax >= 1 ? W(0, 1, t) * mu : 0.0);
  }
  if (lmax >= 2) {
    if (HT) {
      const double* q = coef + kCoef;       // l = 1: P_2
      const double pn = q[0] * mu * pb - q[1] * pa;
      pa = pb; pb = pn;
    }
    const double hp = 0.5 * (1.0 + mu), hm = 0.5 * (1.0 - mu);
    double a0 = 0.0, a1 = hp * hp;          // d^l_22 at l-1, l
    double b0 = 0.0, b1 = hm * hm;          // d^l_2-2
    double c0 = 0.0, c1 = 0.6123724356957945 * (1.0 - mu * mu);   // d^l_20, sqrt(6)/4
    // unrolled twice for one item (measured: 186 -> 164 us for the T+QU N_side 16 Fisher build);
    // with 8 items the weights of two multipoles no longer fit in scalar registers
    constexpr int kLU = IB == 1 ? 2 : 1;
#pragma unroll kLU
    for (int l = 2; l <= lmax; ++l) {
#pragma unroll
      for (int t = 0; t < IB; ++t) {
        if (HT) xtt[t] = fma(W(0, l, t), pb, xtt[t]);
        if (HP) {
          xp[t] = fma(W(1, l, t), a1, xp[t]);
          xm[t] = fma(W(2, l, t), b1, xm[t]);
          xeb[t] = fma(W(5, l, t), b1, xeb[t]);
          if (HT) {
            xte[t] = fma(W(3, l, t), c1, xte[t]);
            xtb[t] = fma(W(4, l, t), c1, xtb[t]);
          }
        }
      }
      if (l < lmax) {
        const double* q = coef + l * kCoef;
        if (HT) {
          const double pn = q[0] * mu * pb - q[1] * pa;
          pa = pb; pb = pn;
        }
        if (HP) {
          const double tq = q[2] * mu;
          const double a2 = (tq - q[3]) * a1 - q[4] * a0;
          const double b2 = (tq + q[3]) * b1 - q[4] * b0;
          a0 = a1; a1 = a2; b0 = b1; b1 = b2;
          if (HT) {
            const double c2 = q[5] * mu * c1 - q[6] * c0;
            c0 = c1; c1 = c2;
          }
        }
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
      // signal + the low-rank noise U U^T (symmetric), once per entry for all items
      const int64_t row = (int64_t)a * npx + i;
      const int64_t col = (int64_t)b * npx + j;
      double uu = 0.0;
      if (live)
        for (int r = 0; r < noise_rank; ++r) uu = fma(noise_U[row * noise_rank + r], noise_U[col * noise_rank + r], uu);
      // at (i, j)
      if (live && !(lower_only && col > row)) {
        const double nv = nvd[a][b];
#pragma unroll
        for (int t = 0; t < IB; ++t) {
          if (t >= cnt) break;
          const double v = (entry(a, b, t) + nv) + uu;
          if (!isfinite(v)) atomicOr(flag, 1);
          C_base[(int64_t)(item0 + t) * c_stride + row * ldc + col] = v;
        }
      }
      // at (j, i) for i > j: entry (b, a) of the mirrored block; in the lower triangle only when b > a
      if (lower_only && b <= a) continue;
      __syncthreads();                       // the previous staged values have been read
      if (live && i > j) {
#pragma unroll
        for (int t = 0; t < IB; ++t) stage[t][tj][ti] = entry(a, b, t);
        stu[tj][ti] = uu;
      }
      __syncthreads();
      if (mlive) {
        const int64_t mrow = (int64_t)b * npx + sj, mcol = (int64_t)a * npx + si;
        const double nv = nvm[a][b];   // off the diagonal: dense noise only
        const double muu = stu[ti][tj];
#pragma unroll
        for (int t = 0; t < IB; ++t) {
          if (t >= cnt) break;
          const double v = (stage[t][ti][tj] + nv) + muu;   // the same order as at (i, j)
          if (!isfinite(v)) atomicOr(flag, 1);
          C_base[(int64_t)(item0 + t) * c_stride + mrow * ldc + mcol] = v;
        }
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
  const int64_t nt = (P.npx + kPT - 1) / kPT;          // tiles per side; the lower triangle of tiles
  if (nt * (nt + 1) / 2 > INT32_MAX) return hipErrorInvalidValue;
  dim3 grid((unsigned)(nt * (nt + 1) / 2), 1, chunks), block(256);
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
