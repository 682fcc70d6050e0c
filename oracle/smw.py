"""Pixel likelihood through the harmonic basis, with multipole switching.

Oracle code: test infrastructure only (see oracle/__init__.py).

Paper Sects. 2.3.2 (Sherman-Morrison-Woodbury identity), 2.3.4 (multipole switching) and 2.6
(pixel-space likelihood).  With V_inf the harmonic operator restricted to the inference window and
Lambda_inf the window's mode covariance,

  C     = N_eff + V_inf^T Lambda_inf V_inf                     (Eq. C_switched)
  N_eff = N + the signal of every multipole held at the fiducial (Eq. N_eff)
  K     = Lambda_inf^-1 + V_inf N_eff^-1 V_inf^T                (Eq. K_kernel, N -> N_eff)
  C^-1  = N_eff^-1 - N_eff^-1 V^T K^-1 V N_eff^-1               (Eq. smw)
  ln|C| = ln|N_eff| + ln|Lambda_inf| + ln|K|                    (Eq. logdet)

and -2 ln L = d^T C^-1 d + ln|C| (Eq. pixel_likelihood, n ln 2 pi left out).

Readings (where the paper leaves the choice open):
* The window is a multipole range [wlo, whi] together with a set of harmonic fields ("T", "E",
  "B"); the paper's switching is by multipole only, which is the case of all the problem's
  fields.  Restricting the fields lets a QU scan that varies only EE keep B in N_eff.
* A spectrum coupling a varied and a fixed field inside the window belongs to neither part of
  the split, so it must vanish there (``check_window``); otherwise N_eff need not be positive
  definite.
* Only the window's entries of a point's spectra among the varied fields are used; every other
  entry is the problem's fiducial value.
"""
import copy

import numpy as np
import scipy.linalg as sla

from . import covariance as cv
from . import healpix

# harmonic fields of each spectrum row (TT, EE, BB, TE, TB, EB)
SPEC_FIELDS = (("T", "T"), ("E", "E"), ("B", "B"), ("T", "E"), ("T", "B"), ("E", "B"))


def check_window(problem, wlo, whi, wfields):
    """Raise ValueError unless [wlo, whi] lies in the problem's range, the fields are among the
    problem's harmonic fields, and no spectrum couples a varied field to a fixed one in the window."""
    present = cv.FIELD_MODES[problem.fields]
    if not (problem.lmin <= wlo <= whi <= problem.lmax):
        raise ValueError("window outside the problem's multipole range")
    if not wfields or any(f not in present for f in wfields):
        raise ValueError("window fields must be a non-empty subset of the problem's fields")
    cl = np.asarray(problem.cl)
    for s, (a, b) in enumerate(SPEC_FIELDS):
        if a not in present or b not in present:
            continue
        if (a in wfields) != (b in wfields) and np.any(cl[s, wlo:whi + 1] != 0.0):
            raise ValueError(f"spectrum {a}{b} couples a varied and a fixed field in the window")


def fixed_spectra(cl, wlo, whi, wfields):
    """The spectra held fixed: the fiducial with the window's entries among varied fields removed
    (those make up Lambda_inf)."""
    out = np.array(cl, dtype=np.float64, copy=True)
    for s, (a, b) in enumerate(SPEC_FIELDS):
        if a in wfields and b in wfields:
            out[s, wlo:whi + 1] = 0.0
    return out


def effective_noise(problem, wlo, whi, wfields):
    """N_eff of Eq. N_eff, assembled by the pixel-pair route of the covariance."""
    p = copy.copy(problem)
    p.cl = fixed_spectra(problem.cl, wlo, whi, wfields)
    return cv.total_covariance(p, route="pairs")


def window_basis(problem, wlo, whi, wfields):
    """V_inf [k_inf][n] (rows: the window's modes) and the list of those modes."""
    th, ph = healpix.active_directions(problem.nside, problem.mask, problem.theta, problem.phi)
    Y, modes = cv.harmonic_basis(th, ph, problem.fields, problem.lmin, problem.lmax)
    sel = [j for j, (f, l, m, cs) in enumerate(modes) if wlo <= l <= whi and f in wfields]
    return Y[:, sel].T, [modes[j] for j in sel]


def smw_minus2lnL(problem, maps, cl_point, wlo, whi, wfields):
    """-2 ln L per map, chi^2 per map and ln|C| with the window's spectra taken from cl_point."""
    check_window(problem, wlo, whi, wfields)
    V, modes = window_basis(problem, wlo, whi, wfields)
    Neff = effective_noise(problem, wlo, whi, wfields)
    Lam = cv.mode_covariance(modes, np.asarray(cl_point, dtype=np.float64), problem.bl, problem.pl)
    d = np.atleast_2d(np.asarray(maps, dtype=np.float64)).T        # [n][nmaps]
    cN = sla.cho_factor(Neff, lower=True)
    Nd = sla.cho_solve(cN, d)                                       # N_eff^-1 d
    NVt = sla.cho_solve(cN, V.T)                                    # N_eff^-1 V^T
    M = V @ NVt
    K = np.linalg.inv(Lam) + M                                      # Eq. K_kernel
    cK = sla.cho_factor(K, lower=True)
    Cinv_d = Nd - NVt @ sla.cho_solve(cK, V @ Nd)                   # Eq. smw applied to d
    chi2 = np.sum(d * Cinv_d, axis=0)
    sign, ld_lam = np.linalg.slogdet(Lam)
    if sign <= 0:
        raise ValueError("the window's mode covariance is not positive definite")
    logdet = (2.0 * np.sum(np.log(np.diag(cN[0]))) + ld_lam
              + 2.0 * np.sum(np.log(np.diag(cK[0]))))               # Eq. logdet
    return chi2 + logdet, chi2, logdet


def window_spectra(problem, cl_point, wlo, whi, wfields):
    """The full spectra whose pixel likelihood the SMW form evaluates: the fiducial outside the
    varied part, cl_point inside it (the input of the direct likelihood for comparisons)."""
    out = np.array(problem.cl, dtype=np.float64, copy=True)
    cp = np.asarray(cl_point, dtype=np.float64)
    for s, (a, b) in enumerate(SPEC_FIELDS):
        if a in wfields and b in wfields:
            out[s, wlo:whi + 1] = cp[s, wlo:whi + 1]
    return out
