// Harmonic basis Y = V^T at the retained pixels (Eqs. S_factored, real_ylm, V_spin2, V_multifield,
// spin_y_def, EB_from_spin).
//
// Columns: [field][l][m: 0, 1c, 1s, 2c, 2s, ...] for fields T, E, B present, l in [lmin, lmax];
// rows: [T | Q | U] pixels.  With sY_lm = sqrt((2l+1)/4pi) d^l_{m,-s}(theta) e^{i m phi},
// E_lm = -(2Y + -2Y)/2 = F+ e^{imphi}, B_lm = i(2Y - -2Y)/2 = i F- e^{imphi},
// Q = sum (a_E E - a_B B), U = sum (a_E B + a_B E), and real modes (sqrt2 Re, sqrt2 Im) for
// m > 0.  One workgroup per pixel; lane m runs the three-term recurrence in l of d^l_{m,0} and
// d^l_{m,+-2}, started at l = max(m, |s|) from the half-angle closed form (log-factorials).
#include "cf_internal.h"

namespace cf {
namespace {

struct Rec {   // state of one Wigner-d recurrence d^l_{M,S} in l
  double M, S, sign, prev, cur;
  int l;       // current l (cur = d^l)
};

__device__ Rec rec_start(int M, int S, double sign, double c, double s) {
  // d^M_{M,S} = (-1)^(M-S) sqrt((2M)! / ((M+S)! (M-S)!)) c^(M+S) s^(M-S)
  double lg = 0.5 * (lgamma(2.0 * M + 1.0) - lgamma((double)(M + S) + 1.0) - lgamma((double)(M - S) + 1.0));
  double v = exp(lg);
  if (M + S) v *= pow(c, (double)(M + S));
  if (M - S) v *= pow(s, (double)(M - S));
  if ((M - S) & 1) v = -v;
  Rec r;
  r.M = M; r.S = S; r.sign = sign; r.prev = 0.0; r.cur = v; r.l = M;
  return r;
}

__device__ void rec_step(Rec& r, double mu) {
  const double l = r.l, M = r.M, S = r.S;
  double nxt;
  if (M == 0.0 && S == 0.0) {
    nxt = ((2.0 * l + 1.0) * mu * r.cur - l * r.prev) / (l + 1.0);
  } else {
    double a = (2.0 * l + 1.0) * (l * (l + 1.0) * mu - M * S);
    double b = (l + 1.0) * sqrt((l * l - M * M) * (l * l - S * S));
    double den = l * sqrt(((l + 1.0) * (l + 1.0) - M * M) * ((l + 1.0) * (l + 1.0) - S * S));
    nxt = (a * r.cur - b * r.prev) / den;
  }
  r.prev = r.cur;
  r.cur = nxt;
  r.l += 1;
}

__global__ __launch_bounds__(128) void k_ybuild(DevProblem P, double* __restrict__ Y, int64_t ldy,
                                                int64_t pgap) {
  const int p = blockIdx.x;
  const double* rec = P.pix + (int64_t)p * kPixRec;
  const double z = rec[8], phi = rec[9];
  const double mu = z;
  const double c = sqrt(fmax(0.0, 0.5 * (1.0 + z))), sh = sqrt(fmax(0.0, 0.5 * (1.0 - z)));
  const int kf = P.kf, lmin = P.lmin, lmax = P.lmax;
  const int fT = 0, fE = P.has_t ? 1 : 0, fB = fE + 1;
  const int64_t rowT = p, rowQ = (P.has_t ? P.npx : 0) + p, rowU = rowQ + P.npx;
  const double sq2 = 1.4142135623730951;
  const int lm2 = lmin * lmin;

  // zero blocks of the block-diagonal basis
  if (P.has_t && P.has_p) {
    double* yt = Y + rowT * ldy;
    double* yq = Y + rowQ * ldy;
    double* yu = Y + rowU * ldy;
    for (int64_t q = threadIdx.x; q < 2 * (int64_t)kf; q += blockDim.x) yt[kf + pgap + q] = 0.0;
    for (int64_t q = threadIdx.x; q < kf; q += blockDim.x) { yq[q] = 0.0; yu[q] = 0.0; }
  }

  for (int m = threadIdx.x; m <= lmax; m += blockDim.x) {
    double sm, cm;
    sincos((double)m * phi, &sm, &cm);
    const int cs0 = (m == 0) ? 0 : 2 * m - 1;
    if (P.has_t) {
      Rec r = rec_start(m, 0, 1.0, c, sh);
      if (m == 0) { r.cur = 1.0; }
      double* y = Y + rowT * ldy + (int64_t)fT * kf;
      for (int l = m;; ) {
        if (l >= lmin) {
          const double v = P.coef[l * kCoef + 7] * r.cur;
          const int64_t col = l * l - lm2 + cs0;
          if (m == 0) y[col] = v;
          else { y[col] = sq2 * v * cm; y[col + 1] = sq2 * v * sm; }
        }
        if (l == lmax) break;
        rec_step(r, mu);
        l = r.l;
      }
    }
    if (P.has_p) {
      // d^l_{m,2} and d^l_{m,-2} mapped to m' >= |s'|: for m < 2, d_{m,2} = (-1)^m d_{2,m}
      // and d_{m,-2} = d_{2,-m}.
      Rec rp, rm;
      if (m >= 2) { rp = rec_start(m, 2, 1.0, c, sh); rm = rec_start(m, -2, 1.0, c, sh); }
      else { rp = rec_start(2, m, (m & 1) ? -1.0 : 1.0, c, sh); rm = rec_start(2, -m, 1.0, c, sh); }
      double* yq = Y + rowQ * ldy;
      double* yu = Y + rowU * ldy;
      const int l0 = m > 2 ? m : 2;
      for (int l = l0;; ) {
        if (l >= lmin) {
          const double nrm = P.coef[l * kCoef + 7];
          const double dp = rp.sign * rp.cur, dm = rm.sign * rm.cur;
          const double Fp = -0.5 * nrm * (dm + dp);
          const double Fm = 0.5 * nrm * (dm - dp);
          const int64_t base = l * l - lm2 + cs0;
          const int64_t ce = (int64_t)fE * kf + pgap + base, cb = (int64_t)fB * kf + pgap + base;
          if (m == 0) {
            // E_l0 = Fp (real), B_l0 = 0
            yq[ce] = Fp; yq[cb] = 0.0;
            yu[ce] = 0.0; yu[cb] = Fp;
          } else {
            const double ec = sq2 * Fp * cm, es = sq2 * Fp * sm;      // E^c, E^s
            const double bc = -sq2 * Fm * sm, bs = sq2 * Fm * cm;     // B^c, B^s
            yq[ce] = ec; yq[ce + 1] = es; yq[cb] = -bc; yq[cb + 1] = -bs;
            yu[ce] = bc; yu[ce + 1] = bs; yu[cb] = ec; yu[cb + 1] = es;
          }
        }
        if (l == lmax) break;
        rec_step(rp, mu);
        rec_step(rm, mu);
        l = rp.l;
      }
    }
  }
}

}  // namespace

hipError_t launch_ybuild(const DevProblem& P, double* Y, int64_t ldy, hipStream_t s, int64_t pgap) {
  if (P.npx <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ybuild, dim3(P.npx), dim3(128), 0, s, P, Y, ldy, pgap);
  return hipGetLastError();
}

}  // namespace cf
