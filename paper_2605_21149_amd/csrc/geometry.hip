// Pixel geometry (HEALPix RING centres, Gorski et al. 2005) and per-multipole tables.
#include "cf_internal.h"
#include <math.h>

namespace cf {
namespace {

// RING pixel index -> (z, phi).  Exact integer ring arithmetic; 1 - z is formed from i^2/(3N^2)
// directly so that sin(theta) keeps full relative precision near the poles.
__device__ void ring_pix2zphi(int64_t p, int nside, double* z, double* omz, double* opz, double* phi) {
  const int64_t N = nside;
  const int64_t npix = 12 * N * N;
  const int64_t ncap = 2 * N * (N - 1);
  const double pi = 3.14159265358979323846;
  if (p < ncap) {                                   // north polar cap
    int64_t i = (int64_t)((1.0 + sqrt(1.0 + 2.0 * (double)p)) * 0.5);
    while (2 * i * (i - 1) > p) --i;
    while (2 * (i + 1) * i <= p) ++i;
    int64_t j = p - 2 * i * (i - 1) + 1;
    double t = (double)(i * i) / (3.0 * (double)(N * N));
    *omz = t; *opz = 2.0 - t; *z = 1.0 - t;
    *phi = (j - 0.5) * pi / (2.0 * (double)i);
  } else if (p < npix - ncap) {                     // equatorial belt
    int64_t q = p - ncap;
    int64_t i = q / (4 * N) + N;
    int64_t j = q % (4 * N) + 1;
    int64_t s = (i - N + 1) & 1;
    double zz = 4.0 / 3.0 - 2.0 * (double)i / (3.0 * (double)N);
    *z = zz; *omz = 1.0 - zz; *opz = 1.0 + zz;
    *phi = ((double)j - 1.0 + 0.5 * (double)s) * pi / (2.0 * (double)N);
  } else {                                          // south polar cap (mirror)
    int64_t q = npix - p;                           // 1-based from the end
    int64_t i = (int64_t)((1.0 + sqrt(2.0 * (double)q - 1.0)) * 0.5);
    while (2 * i * (i - 1) >= q) --i;
    while (2 * (i + 1) * i < q) ++i;
    int64_t j = 4 * i + 1 - (q - 2 * i * (i - 1));
    double t = (double)(i * i) / (3.0 * (double)(N * N));
    *opz = t; *omz = 2.0 - t; *z = t - 1.0;
    *phi = (j - 0.5) * pi / (2.0 * (double)i);
  }
}

__global__ void k_geometry(const int* ring_idx, int nside, const double* theta, const double* phi_in,
                           int npx, double* pix) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npx) return;
  double z, st, phi;
  if (nside > 0) {
    double omz, opz;
    ring_pix2zphi(ring_idx[p], nside, &z, &omz, &opz, &phi);
    st = sqrt(omz * opz);
  } else {
    double th = theta[p];
    phi = phi_in[p];
    z = cos(th);
    st = sin(th);
  }
  double sp, cp;
  sincos(phi, &sp, &cp);
  double* r = pix + (int64_t)p * kPixRec;
  r[0] = st * cp; r[1] = st * sp; r[2] = z;          // n
  r[3] = z * cp;  r[4] = z * sp;  r[5] = -st;        // e_theta
  r[6] = -sp;     r[7] = cp;                         // e_phi (z component 0)
  r[8] = z;       r[9] = phi;
}

// Per-multipole tables: weights c^XY_l (in the order TT, EE + BB, EE - BB, TE, TB, EB), window
// W_l, mode covariance C^XY_l W_l, recurrence coefficients.  One thread per (item, l); items are scan points sharing one problem.
__global__ void k_tables(const double* cl, const double* bl, const double* pl, int lmin, int lmax,
                         int64_t cl_stride, int64_t cl_ld, double* cw, double* wl, double* lam,
                         double* coef, const int64_t* i0p, int nitems, int inter) {
  const int L = lmax + 1;
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  int item = blockIdx.y;
  if (l >= L) return;
  const double pi = 3.14159265358979323846;
  double b = bl ? bl[l] : 1.0;
  double w = pl ? pl[l] : 1.0;
  double W = b * b * w * w;
  double f = (2.0 * l + 1.0) / (4.0 * pi) * W;
  const bool real = item < nitems;                   // false: zero padding of the last chunk
  const double* c = cl + (item + (i0p ? *i0p : 0)) * cl_stride;
  double v[6];
  for (int x = 0; x < 6; ++x) v[x] = real ? c[(int64_t)x * cl_ld + l] : 0.0;
  for (int x = 0; x < 6; ++x) {
    if (cw) {
      // the covariance assembly takes the EE and BB weights as their sum and difference
      const double u = x == 1 ? v[1] + v[2] : (x == 2 ? v[1] - v[2] : v[x]);
      const int64_t at = inter > 1 ? (((int64_t)(item / inter) * L + l) * 6 + x) * inter + item % inter
                                   : (int64_t)item * 6 * L + x * L + l;
      cw[at] = (l >= lmin) ? f * u : 0.0;
    }
    if (lam && real) lam[(int64_t)item * 6 * L + x * L + l] = (l >= lmin) ? W * v[x] : 0.0;
  }
  if (item == 0) {
    if (wl) wl[l] = W;
    if (coef) {
      double dl = (double)l;
      double* q = coef + (int64_t)l * kCoef;
      // Legendre: (l+1) P_{l+1} = (2l+1) mu P_l - l P_{l-1}
      q[0] = (2.0 * dl + 1.0) / (dl + 1.0);
      q[1] = dl / (dl + 1.0);
      // d^l_{2,+-2}: l((l+1)^2-4) d^{l+1} = (2l+1)(l(l+1) mu -+ 4) d^l - (l+1)(l^2-4) d^{l-1}
      if (l >= 2) {
        double den = dl * ((dl + 1.0) * (dl + 1.0) - 4.0);
        q[2] = (2.0 * dl + 1.0) * dl * (dl + 1.0) / den;
        q[3] = 4.0 * (2.0 * dl + 1.0) / den;
        q[4] = (dl + 1.0) * (dl * dl - 4.0) / den;
        // d^l_{20}: sqrt((l+1)^2-4) d^{l+1} = (2l+1) mu d^l - sqrt(l^2-4) d^{l-1}
        double s1 = sqrt((dl + 1.0) * (dl + 1.0) - 4.0);
        q[5] = (2.0 * dl + 1.0) / s1;
        q[6] = sqrt(dl * dl - 4.0) / s1;
      } else {
        q[2] = q[3] = q[4] = q[5] = q[6] = 0.0;
      }
      q[7] = sqrt((2.0 * dl + 1.0) / (4.0 * pi));
    }
  }
}

}  // namespace

hipError_t launch_geometry(const int* ring_idx, int nside, const double* theta, const double* phi,
                           int npx, double* pix, hipStream_t s) {
  if (npx <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_geometry, dim3((npx + 255) / 256), dim3(256), 0, s, ring_idx, nside, theta,
                     phi, npx, pix);
  return hipGetLastError();
}

hipError_t launch_tables(const double* cl, const double* bl, const double* pl, int lmin, int lmax,
                         int nitems, int64_t cl_stride, int64_t cl_ld, double* cw, double* wl,
                         double* lam, double* coef, hipStream_t s, const int64_t* i0p, int interleave) {
  int L = lmax + 1;
  if (interleave < 1 || nitems <= 0) return hipErrorInvalidValue;
  const int padded = (nitems + interleave - 1) / interleave * interleave;
  hipLaunchKernelGGL(k_tables, dim3((L + 127) / 128, padded), dim3(128), 0, s, cl, bl, pl, lmin,
                     lmax, cl_stride, cl_ld, cw, wl, lam, coef, i0p, nitems, interleave);
  return hipGetLastError();
}

}  // namespace cf
