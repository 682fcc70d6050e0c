"""Pixel covariance C = S + N for spin-0 and spin-2 fields (Eqs. total_cov, signal_cov; App. A).

Oracle code: test infrastructure only (see oracle/__init__.py).

Two independent routes to S:

* ``signal_pairs``: for every pixel pair, the correlation functions in the frame
  of the great circle through the pair (Legendre P_l for TT, d^l_{22},
  d^l_{2,-2} for Q/U, d^l_{20} for T x Q/U), rotated to each pixel's local
  (theta, phi) frame with the angles psi_p, psi_p' between the local meridian
  and that great circle (App. A.4).  The recurrences here are written for the
  three fixed (m, s) pairs and share nothing with ``wigner.py``.
* ``signal_harmonic``: S = Y Lambda Y^T with Y = V^T the real harmonic basis at
  the active pixels (Eq. S_factored): real Y_lm from scipy for T (Eq. real_ylm)
  and the E/B functions of Eq. EB_from_spin built from spin_y_def with
  ``wigner.wigner_d`` for Q/U.

Conventions (readings of the paper where it leaves the choice open):
* data order [T | Q | U] over the same active pixels (Eqs. V_multifield);
* (Q + iU) = sum a_{2,lm} 2Y_lm, (Q - iU) = sum a_{-2,lm} -2Y_lm with
  a_E = -(a_2 + a_-2)/2, a_B = i (a_2 - a_-2)/2, so that
  Q = sum (a_E E_lm - a_B B_lm) and U = sum (a_E B_lm + a_B E_lm) with the
  E_lm, B_lm of Eq. EB_from_spin;
* real modes: for m > 0 the pair (sqrt2 Re X_lm, sqrt2 Im X_lm), for m = 0 X_l0;
* per-multipole weight c^XY_l = (2l+1)/(4 pi) C^XY_l W_l, W_l = B_l^2 p_l^2.
"""
import numpy as np
from scipy.special import sph_harm_y

from . import healpix
from .wigner import wigner_d

SPECS = ("TT", "EE", "BB", "TE", "TB", "EB")
FIELD_MAPS = {"T": ("T",), "QU": ("Q", "U"), "TQU": ("T", "Q", "U")}
FIELD_MODES = {"T": ("T",), "QU": ("E", "B"), "TQU": ("T", "E", "B")}


def window(bl, pl):
    """W_l = B_l^2 p_l^2 (Eq. signal_cov)."""
    return np.asarray(bl) ** 2 * np.asarray(pl) ** 2


def ell_weights(cl, bl, pl, lmin, lmax):
    """c^XY_l = (2l+1)/(4 pi) C^XY_l W_l for l in [lmin, lmax], zero elsewhere; [6][lmax+1]."""
    ell = np.arange(lmax + 1)
    w = (2 * ell + 1) / (4 * np.pi) * window(bl[:lmax + 1], pl[:lmax + 1])
    c = np.asarray(cl, dtype=np.float64)[:, :lmax + 1] * w[None, :]
    c[:, :lmin] = 0.0
    return c


# ---------------------------------------------------------------------------
# pair route
# ---------------------------------------------------------------------------
def pair_functions(mu, lmin, lmax):
    """P_l(mu), d^l_22(mu), d^l_2-2(mu), d^l_20(mu) for l = 0..lmax, each [lmax+1, len(mu)].

    Legendre: (l+1) P_{l+1} = (2l+1) mu P_l - l P_{l-1}.
    Spin-2, started at l = 2 from d^2_22 = ((1+mu)/2)^2, d^2_2-2 = ((1-mu)/2)^2,
    d^2_20 = sqrt(6)/4 (1 - mu^2):
      l((l+1)^2-4) d^{l+1}_{2,+-2} = (2l+1)(l(l+1)mu -+ 4) d^l - (l+1)(l^2-4) d^{l-1}
      sqrt((l+1)^2-4) d^{l+1}_20    = (2l+1) mu d^l_20 - sqrt(l^2-4) d^{l-1}_20
    """
    mu = np.asarray(mu, dtype=np.float64)
    L = lmax + 1
    P = np.zeros((L,) + mu.shape)
    d22 = np.zeros_like(P)
    d2m2 = np.zeros_like(P)
    d20 = np.zeros_like(P)
    P[0] = 1.0
    if lmax >= 1:
        P[1] = mu
    for l in range(1, lmax):
        P[l + 1] = ((2 * l + 1) * mu * P[l] - l * P[l - 1]) / (l + 1)
    if lmax >= 2:
        d22[2] = ((1 + mu) / 2) ** 2
        d2m2[2] = ((1 - mu) / 2) ** 2
        d20[2] = np.sqrt(6.0) / 4.0 * (1 - mu * mu)
    for l in range(2, lmax):
        den = l * ((l + 1) ** 2 - 4)
        d22[l + 1] = ((2 * l + 1) * (l * (l + 1) * mu - 4) * d22[l] - (l + 1) * (l * l - 4) * d22[l - 1]) / den
        d2m2[l + 1] = ((2 * l + 1) * (l * (l + 1) * mu + 4) * d2m2[l] - (l + 1) * (l * l - 4) * d2m2[l - 1]) / den
        d20[l + 1] = ((2 * l + 1) * mu * d20[l] - np.sqrt(l * l - 4.0) * d20[l - 1]) / np.sqrt((l + 1) ** 2 - 4.0)
    return P, d22, d2m2, d20


def local_frames(theta, phi):
    """Unit vector n, e_theta, e_phi at each direction."""
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    n = np.stack([st * cp, st * sp, ct], axis=-1)
    et = np.stack([ct * cp, ct * sp, -st], axis=-1)
    ep = np.stack([-sp, cp, np.zeros_like(phi)], axis=-1)
    return n, et, ep


def rotation_angle(n_other, et, ep, tiny=1e-12):
    """Angle psi at a pixel from its local meridian (e_theta) to the great circle toward
    ``n_other``, measured toward e_phi.  Coincident or antipodal pairs (no unique great
    circle) take the meridian, psi = 0 (App. A.4)."""
    a = np.sum(n_other * et, axis=-1)
    b = np.sum(n_other * ep, axis=-1)
    degenerate = a * a + b * b < tiny
    a = np.where(degenerate, 1.0, a)
    b = np.where(degenerate, 0.0, b)
    return np.arctan2(b, a)


def signal_pairs(theta, phi, fields, cl, bl, pl, lmin, lmax, rows=None):
    """Signal covariance by pixel pairs; returns [n][n] (or the requested row block).

    ``rows``: optional array of active-pixel indices i; the result then holds the
    rows (field, i) for those pixels against every column, as [nmaps*len(rows)][n].
    """
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    npx = theta.size
    maps = FIELD_MAPS[fields]
    nm = len(maps)
    c = ell_weights(cl, bl, pl, lmin, lmax)
    idx_i = np.arange(npx) if rows is None else np.asarray(rows)
    n, et, ep = local_frames(theta, phi)
    ni, eti, epi = n[idx_i], et[idx_i], ep[idx_i]
    mu = np.clip(ni @ n.T, -1.0, 1.0)                      # [ri][npx]
    P, d22, d2m2, d20 = pair_functions(mu, lmin, lmax)
    xi_tt = np.tensordot(c[0], P, axes=(0, 0))
    xi_p = np.tensordot(c[1] + c[2], d22, axes=(0, 0))
    xi_m = np.tensordot(c[1] - c[2], d2m2, axes=(0, 0))
    xi_eb = np.tensordot(c[5], d2m2, axes=(0, 0))
    xi_te = np.tensordot(c[3], d20, axes=(0, 0))
    xi_tb = np.tensordot(c[4], d20, axes=(0, 0))
    # psi_i: at pixel i toward j ; psi_j: at pixel j toward i
    psi_i = rotation_angle(n[None, :, :], eti[:, None, :], epi[:, None, :])
    psi_j = rotation_angle(ni[:, None, :], et[None, :, :], ep[None, :, :])
    # <P_i P_j*> = e^{2i(psi_i - psi_j)} xi_+ ; <P_i P_j> = e^{2i(psi_i + psi_j)} (xi_- + 2i xi_EB)
    ppc = np.exp(2j * (psi_i - psi_j)) * xi_p
    pp = np.exp(2j * (psi_i + psi_j)) * (xi_m + 2j * xi_eb)
    qq = 0.5 * (ppc.real + pp.real)
    uu = 0.5 * (ppc.real - pp.real)
    qu = 0.5 * (pp.imag - ppc.imag)          # <Q_i U_j>
    uq = 0.5 * (pp.imag + ppc.imag)          # <U_i Q_j>
    # <T_i P_j*> = -e^{-2i psi_j} (xi_TE - i xi_TB) = <T_i Q_j> - i <T_i U_j>
    tpc = -np.exp(-2j * psi_j) * (xi_te - 1j * xi_tb)
    tq, tu = tpc.real, -tpc.imag
    # <P_i T_j> = -e^{2i psi_i} (xi_TE + i xi_TB) = <Q_i T_j> + i <U_i T_j>
    pt = -np.exp(2j * psi_i) * (xi_te + 1j * xi_tb)
    qt, ut = pt.real, pt.imag
    blocks = {("T", "T"): xi_tt, ("Q", "Q"): qq, ("U", "U"): uu, ("Q", "U"): qu,
              ("U", "Q"): uq, ("T", "Q"): tq, ("T", "U"): tu, ("Q", "T"): qt, ("U", "T"): ut}
    ri = idx_i.size
    S = np.zeros((nm * ri, nm * npx))
    for a, fa in enumerate(maps):
        for b, fb in enumerate(maps):
            S[a * ri:(a + 1) * ri, b * npx:(b + 1) * npx] = blocks[(fa, fb)]
    return S


# ---------------------------------------------------------------------------
# harmonic route
# ---------------------------------------------------------------------------
def mode_index(fields, lmin, lmax):
    """List of (mode_field, l, m, cs) per column of Y, ordered [field][l][m: 0, 1c, 1s, ...]."""
    out = []
    for f in FIELD_MODES[fields]:
        for l in range(lmin, lmax + 1):
            out.append((f, l, 0, 0))
            for m in range(1, l + 1):
                out.append((f, l, m, 0))
                out.append((f, l, m, 1))
    return out


def harmonic_basis(theta, phi, fields, lmin, lmax):
    """Y = V^T, [n][n_modes]: real harmonics at the active pixels (Eqs. real_ylm, V_spin2,
    V_multifield, spin_y_def, EB_from_spin) with (2l+1)/(4 pi) absorbed."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    npx = theta.size
    maps = FIELD_MAPS[fields]
    modes = mode_index(fields, lmin, lmax)
    col = {key: j for j, key in enumerate(modes)}
    Y = np.zeros((len(maps) * npx, len(modes)))
    row0 = {f: k * npx for k, f in enumerate(maps)}
    sq2 = np.sqrt(2.0)
    if "T" in maps:
        for l in range(lmin, lmax + 1):
            for m in range(0, l + 1):
                y = sph_harm_y(l, m, theta, phi)
                r = slice(row0["T"], row0["T"] + npx)
                if m == 0:
                    Y[r, col[("T", l, 0, 0)]] = y.real
                else:
                    Y[r, col[("T", l, m, 0)]] = sq2 * y.real
                    Y[r, col[("T", l, m, 1)]] = sq2 * y.imag
    if "Q" in maps:
        rq = slice(row0["Q"], row0["Q"] + npx)
        ru = slice(row0["U"], row0["U"] + npx)
        for m in range(0, lmax + 1):
            dp = wigner_d(lmax, m, 2, theta)    # d^l_{m,2}
            dm = wigner_d(lmax, m, -2, theta)   # d^l_{m,-2}
            for l in range(max(lmin, m, 2), lmax + 1):
                norm = np.sqrt((2 * l + 1) / (4 * np.pi))
                # E_lm = Fp e^{imphi}, B_lm = i Fm e^{imphi}  (Eqs. spin_y_def, EB_from_spin)
                Fp = -0.5 * norm * (dm[l] + dp[l])
                Fm = 0.5 * norm * (dm[l] - dp[l])
                E = Fp * np.exp(1j * m * phi)
                B = 1j * Fm * np.exp(1j * m * phi)
                if m == 0:
                    parts = [(0, E.real, B.real)]
                else:
                    parts = [(0, sq2 * E.real, sq2 * B.real), (1, sq2 * E.imag, sq2 * B.imag)]
                for cs, e, b in parts:
                    ce, cb = col[("E", l, m, cs)], col[("B", l, m, cs)]
                    Y[rq, ce] = e          # Q <- a_E E
                    Y[rq, cb] = -b         # Q <- -a_B B
                    Y[ru, ce] = b          # U <- a_E B
                    Y[ru, cb] = e          # U <- a_B E
    return Y, modes


def mode_covariance(modes, cl, bl, pl):
    """Lambda (Eqs. Lambda_spin2, Lambda_TEB): block-diagonal in (l, m, cs), entries C^XY_l W_l."""
    W = window(bl, pl)
    k = len(modes)
    Lam = np.zeros((k, k))
    pos = {}
    for j, (f, l, m, cs) in enumerate(modes):
        pos.setdefault((l, m, cs), {})[f] = j
    name = {("T", "T"): 0, ("E", "E"): 1, ("B", "B"): 2, ("T", "E"): 3, ("E", "T"): 3,
            ("T", "B"): 4, ("B", "T"): 4, ("E", "B"): 5, ("B", "E"): 5}
    for (l, m, cs), fmap in pos.items():
        for fa, ja in fmap.items():
            for fb, jb in fmap.items():
                Lam[ja, jb] = cl[name[(fa, fb)]][l] * W[l]
    return Lam


def signal_harmonic(theta, phi, fields, cl, bl, pl, lmin, lmax):
    Y, modes = harmonic_basis(theta, phi, fields, lmin, lmax)
    Lam = mode_covariance(modes, cl, bl, pl)
    return Y @ Lam @ Y.T


def total_covariance(problem, route="pairs"):
    """C = S + N (Eq. total_cov) for an ``inputs.Problem``-like object."""
    th, ph = healpix.active_directions(problem.nside, problem.mask, problem.theta, problem.phi)
    if route == "pairs":
        S = signal_pairs(th, ph, problem.fields, problem.cl, problem.bl, problem.pl,
                         problem.lmin, problem.lmax)
    else:
        S = signal_harmonic(th, ph, problem.fields, problem.cl, problem.bl, problem.pl,
                            problem.lmin, problem.lmax)
    return S + problem.noise_matrix()
