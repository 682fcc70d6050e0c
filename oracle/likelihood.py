"""Gaussian pixel likelihood -2 ln L = d^T C^-1 d + ln|C| (Eq. pixel_likelihood).

Oracle code: test infrastructure only (see oracle/__init__.py).
The constant n ln(2 pi) is left out.
"""
import numpy as np
import scipy.linalg as sla

from . import covariance as cv


def chi2_logdet(C, maps):
    """chi^2_j = ||L^-1 d_j||^2 for each map and ln|C| = 2 sum ln L_ii, C = L L^T."""
    L = sla.cholesky(C, lower=True)
    u = sla.solve_triangular(L, np.atleast_2d(maps).T, lower=True)
    return np.sum(u * u, axis=0), 2.0 * np.sum(np.log(np.diag(L)))


def minus2lnL(problem, maps, cl=None):
    """[-2 ln L per map], chi^2 per map and ln|C| for the problem (optionally other spectra)."""
    if cl is not None:
        problem = _with_cl(problem, cl)
    C = cv.total_covariance(problem)
    chi2, logdet = chi2_logdet(C, maps)
    return chi2 + logdet, chi2, logdet


def _with_cl(problem, cl):
    import copy
    p = copy.copy(problem)
    p.cl = np.asarray(cl, dtype=np.float64)
    return p


def scan(problem, maps, cl_points):
    """-2 ln L over parameter points: [npoints][nmaps] plus ln|C| per point."""
    m2 = np.zeros((len(cl_points), np.atleast_2d(maps).shape[0]))
    ld = np.zeros(len(cl_points))
    for i, cl in enumerate(cl_points):
        m2[i], _, ld[i] = minus2lnL(problem, maps, cl)
    return m2, ld
