"""Small Wigner d-functions d^l_{m,s}(theta) (App. A.3 of the paper).

Oracle code: test infrastructure only (see oracle/__init__.py).

Computed by the three-term recurrence in l at fixed (m, s).  Any requested
(m, s) is first mapped into the range m >= |s|, m >= 0 with the symmetries
d^l_{m,s} = (-1)^(m-s) d^l_{s,m} = (-1)^(m-s) d^l_{-m,-s}; the recurrence is
started at l = m from the closed form in half angles, whose factorials are
evaluated through their logarithms.
"""
import math

import numpy as np


def _canonical(m, s):
    """Return (sign, M, S) with d^l_{m,s} = sign * d^l_{M,S}, M >= |S|, M >= 0."""
    sign = 1
    if abs(m) < abs(s):                      # d_{m,s} = (-1)^(m-s) d_{s,m}
        sign *= (-1) ** ((m - s) & 1)
        m, s = s, m
    if m < 0:                                # d_{m,s} = (-1)^(m-s) d_{-m,-s}
        sign *= (-1) ** ((m - s) & 1)
        m, s = -m, -s
    return sign, m, s


def wigner_d(lmax, m, s, theta):
    """Array [lmax+1, len(theta)] of d^l_{m,s}(theta); rows l < max(|m|,|s|) are zero."""
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    out = np.zeros((lmax + 1, theta.size))
    sign, M, S = _canonical(m, s)
    if M > lmax:
        return out
    mu = np.cos(theta)
    if M == 0:  # then S == 0: Legendre polynomials
        out[0] = 1.0
        if lmax >= 1:
            out[1] = mu
        for l in range(1, lmax):
            out[l + 1] = ((2 * l + 1) * mu * out[l] - l * out[l - 1]) / (l + 1)
        return sign * out
    # closed form at l = M:  d^M_{M,S} = (-1)^(M-S) sqrt((2M)!/((M+S)!(M-S)!)) c^(M+S) s^(M-S)
    c = np.cos(0.5 * theta)
    sn = np.sin(0.5 * theta)
    lognorm = 0.5 * (math.lgamma(2 * M + 1) - math.lgamma(M + S + 1) - math.lgamma(M - S + 1))
    with np.errstate(divide="ignore"):
        logc = np.where(c > 0, np.log(np.abs(c)), -np.inf)
        logs = np.where(sn > 0, np.log(np.abs(sn)), -np.inf)
    logv = lognorm + (M + S) * logc if M + S else np.full_like(theta, lognorm)
    logv = logv + ((M - S) * logs if M - S else 0.0)
    out[M] = (-1) ** ((M - S) & 1) * np.exp(logv)
    # l d^{l+1} sqrt(((l+1)^2-M^2)((l+1)^2-S^2))
    #    = (2l+1)(l(l+1) mu - M S) d^l - (l+1) sqrt((l^2-M^2)(l^2-S^2)) d^{l-1}
    for l in range(M, lmax):
        a = (2 * l + 1) * (l * (l + 1) * mu - M * S)
        b = (l + 1) * math.sqrt((l * l - M * M) * (l * l - S * S))
        den = l * math.sqrt(((l + 1) ** 2 - M * M) * ((l + 1) ** 2 - S * S))
        prev = out[l - 1] if l >= 1 else 0.0
        out[l + 1] = (a * out[l] - b * prev) / den
    return sign * out
