"""Fisher matrix, QML quadratic forms, noise bias and deconvolved spectra.

Oracle code: test infrastructure only (see oracle/__init__.py).

Parameters are (spectrum XY, bin b) pairs, index s * n_b + b with s running over
the requested spectra in TT, EE, BB, TE, TB, EB order.  The bin derivative is
P_b = sum_{l in b} dC/dC^XY_l, so W_l enters once (reading of the binning of
Sect. 2.4; pinned by the binning identity F_binned = P F P^T).

Two routes:
* ``*_dense``: the definitions in pixel space, Eqs. fisher, P_ell, q_ell,
  noise_bias (derivative matrices built with the pair route);
* ``*_harmonic``: Z = Y^T C^-1 Y (Eq. projected_inv, computed directly) with the
  COO trace of Eq. sparse_trace, w = Y^T C^-1 d (Eq. weighted_data) and
  Eq. q_harmonic; the noise bias as 1/2 tr[E_b (Z - Z Lambda Z)], which equals
  Eq. noise_bias because Y^T C^-1 N C^-1 Y = Z - Z Lambda Z when the signal band
  is the analysis window.
"""
import numpy as np
import scipy.linalg as sla

from . import covariance as cv
from . import healpix

SPECS = cv.SPECS
_PAIRS = {"TT": (("T", "T"),), "EE": (("E", "E"),), "BB": (("B", "B"),),
          "TE": (("T", "E"), ("E", "T")), "TB": (("T", "B"), ("B", "T")),
          "EB": (("E", "B"), ("B", "E"))}


def parameters(spectra, lo, hi):
    """[(spec, l_lo, l_hi)] in Fisher index order s * n_b + b."""
    order = [s for s in SPECS if s in spectra]
    return [(s, int(a), int(b)) for s in order for a, b in zip(lo, hi)]


def _directions(problem):
    return healpix.active_directions(problem.nside, problem.mask, problem.theta, problem.phi)


def derivative_dense(problem, spec, l_lo, l_hi):
    """P_b = sum_{l in [l_lo, l_hi]} dC/dC^spec_l (Eq. P_ell and its spin-2 extension)."""
    th, ph = _directions(problem)
    unit = np.zeros((6, problem.lmax + 1))
    unit[SPECS.index(spec), l_lo:l_hi + 1] = 1.0
    return cv.signal_pairs(th, ph, problem.fields, unit, problem.bl, problem.pl,
                           problem.lmin, problem.lmax)


def fisher_dense(problem, spectra, lo, hi, C=None):
    """F_AB = 1/2 tr[C^-1 P_A C^-1 P_B] (Eq. fisher)."""
    if C is None:
        C = cv.total_covariance(problem)
    fac = sla.cho_factor(C, lower=True)
    pars = parameters(spectra, lo, hi)
    CiP = [sla.cho_solve(fac, derivative_dense(problem, *p)) for p in pars]
    k = len(pars)
    F = np.zeros((k, k))
    for a in range(k):
        for b in range(k):
            F[a, b] = 0.5 * np.sum(CiP[a] * CiP[b].T)     # tr[A B] = sum A * B^T
    return F


def quadratic_dense(problem, spectra, lo, hi, maps, C=None):
    """y_A = 1/2 d^T C^-1 P_A C^-1 d (the data term of Eq. q_ell) for each map; [nmaps][k]."""
    if C is None:
        C = cv.total_covariance(problem)
    fac = sla.cho_factor(C, lower=True)
    x = sla.cho_solve(fac, np.atleast_2d(maps).T)          # C^-1 d, [n][nmaps]
    pars = parameters(spectra, lo, hi)
    y = np.zeros((x.shape[1], len(pars)))
    for a, p in enumerate(pars):
        P = derivative_dense(problem, *p)
        y[:, a] = 0.5 * np.sum(x * (P @ x), axis=0)
    return y


def bias_dense(problem, spectra, lo, hi, C=None):
    """b_A = 1/2 tr[C^-1 P_A C^-1 N] (Eq. noise_bias)."""
    if C is None:
        C = cv.total_covariance(problem)
    fac = sla.cho_factor(C, lower=True)
    CiN = sla.cho_solve(fac, problem.noise_matrix())
    pars = parameters(spectra, lo, hi)
    out = np.zeros(len(pars))
    for a, p in enumerate(pars):
        CiP = sla.cho_solve(fac, derivative_dense(problem, *p))
        out[a] = 0.5 * np.sum(CiP * CiN.T)
    return out


def cross_dense(problem1, problem2, spectra, lo, hi, maps1, maps2):
    """Cross-QML of two data sets filtered independently (Eq. q_cross):
      q_A = 1/2 d1^T C1^-1 P_A C2^-1 d2     (per map pair j: maps1[j], maps2[j])
      W_AB = 1/2 tr[C1^-1 P_A C2^-1 P_B]    (the mode-mixing matrix beside Eq. q_cross)
      C_hat = W^-1 q                        (deconvolved as in Eq. qml_estimate; no noise bias)
    The two problems share geometry, spectra, beam and window (so P_A and S are common) and differ
    in their noise.  Returns (q [nmaps][k], W [k][k], C_hat [nmaps][k])."""
    f1 = sla.cho_factor(cv.total_covariance(problem1), lower=True)
    f2 = sla.cho_factor(cv.total_covariance(problem2), lower=True)
    x1 = sla.cho_solve(f1, np.atleast_2d(maps1).T)          # C1^-1 d1
    x2 = sla.cho_solve(f2, np.atleast_2d(maps2).T)          # C2^-1 d2
    pars = parameters(spectra, lo, hi)
    P = [derivative_dense(problem1, *p) for p in pars]
    A1 = [sla.cho_solve(f1, Pa) for Pa in P]                # C1^-1 P_A
    A2 = [sla.cho_solve(f2, Pa) for Pa in P]                # C2^-1 P_A
    k = len(pars)
    q = np.zeros((x1.shape[1], k))
    W = np.zeros((k, k))
    for a in range(k):
        q[:, a] = 0.5 * np.sum(x1 * (P[a] @ x2), axis=0)
        for b in range(k):
            W[a, b] = 0.5 * np.sum(A1[a] * A2[b].T)         # tr[C1^-1 P_a C2^-1 P_b]
    chat = np.linalg.solve(W, q.T).T
    return q, W, chat


def joint_dense(problem1, problem2, spectra, lo, hi, maps1, maps2, N12=None, s12=1.0):
    """QML of the joint data vector d = (d1, d2) of two data sets of one sky (Eq. C_joint):
      C_j = [[S + N1, s12 S + N12], [s12 S + N12^T, S + N2]],   N_j = [[N1, N12], [N12^T, N2]],
      P_A^j = dC_j/dC_A = [[P_A, s12 P_A], [s12 P_A, P_A]],
    then the standard estimator on the 2n-dimensional system (Eqs. fisher, q_ell, noise_bias,
    qml_estimate): F_AB = 1/2 tr[C_j^-1 P_A^j C_j^-1 P_B^j], y_A = 1/2 d^T C_j^-1 P_A^j C_j^-1 d,
    b_A = 1/2 tr[C_j^-1 P_A^j C_j^-1 N_j], C_hat = F^-1 (y - b).  Both data sets see the same
    signal (s12 = 1, the equation as written); s12 = 0 decouples the two skies (a test case).
    Geometry, spectra, beam and window come from problem1; problem2 contributes its noise N2;
    N12[i][j] = Cov(n1_i, n2_j) (None: independent noise).  Returns dict(F, y, bias, chat)."""
    th, ph = _directions(problem1)
    S = cv.signal_pairs(th, ph, problem1.fields, problem1.cl, problem1.bl, problem1.pl,
                        problem1.lmin, problem1.lmax)
    n = S.shape[0]
    X = np.zeros((n, n)) if N12 is None else np.asarray(N12, dtype=np.float64)
    Nj = np.block([[problem1.noise_matrix(), X], [X.T, problem2.noise_matrix()]])
    Cj = np.block([[S, s12 * S], [s12 * S, S]]) + Nj
    fac = sla.cho_factor(Cj, lower=True)
    pars = parameters(spectra, lo, hi)
    Pj = []
    for p in pars:
        P = derivative_dense(problem1, *p)
        Pj.append(np.block([[P, s12 * P], [s12 * P, P]]))
    CiP = [sla.cho_solve(fac, P) for P in Pj]
    k = len(pars)
    F = np.zeros((k, k))
    for a in range(k):
        for b in range(k):
            F[a, b] = 0.5 * np.sum(CiP[a] * CiP[b].T)
    d = np.hstack([np.atleast_2d(maps1), np.atleast_2d(maps2)])     # [nmaps][2n]
    x = sla.cho_solve(fac, d.T)
    y = np.zeros((d.shape[0], k))
    CiN = sla.cho_solve(fac, Nj)
    bias = np.zeros(k)
    for a in range(k):
        y[:, a] = 0.5 * np.sum(x * (Pj[a] @ x), axis=0)
        bias[a] = 0.5 * np.sum(CiP[a] * CiN.T)
    return {"F": F, "y": y, "bias": bias, "chat": deconvolve(F, y - bias[None, :])}


# ---------------------------------------------------------------------------
# harmonic (Z) route
# ---------------------------------------------------------------------------
def coo_derivatives(problem, modes, spectra, lo, hi):
    """E_A as COO triplets (r, c, v): v = W_l at the (field pair, l, m) entries of A."""
    W = cv.window(problem.bl, problem.pl)
    col = {key: j for j, key in enumerate(modes)}
    out = []
    for spec, a, b in parameters(spectra, lo, hi):
        r, c, v = [], [], []
        for l in range(a, b + 1):
            for fa, fb in _PAIRS[spec]:
                for m in range(0, l + 1):
                    for cs in ((0,) if m == 0 else (0, 1)):
                        r.append(col[(fa, l, m, cs)])
                        c.append(col[(fb, l, m, cs)])
                        v.append(W[l])
        out.append((np.array(r), np.array(c), np.array(v)))
    return out


def projected_inverse(problem, C=None):
    """Z = Y^T C^-1 Y (Eq. projected_inv) with Y, the mode list, and the Cholesky factor of C."""
    if C is None:
        C = cv.total_covariance(problem)
    th, ph = _directions(problem)
    Y, modes = cv.harmonic_basis(th, ph, problem.fields, problem.lmin, problem.lmax)
    fac = sla.cho_factor(C, lower=True)
    Z = Y.T @ sla.cho_solve(fac, Y)
    return Z, Y, modes, fac


def fisher_from_z(Z, coo):
    """Eq. sparse_trace: F_AB = 1/2 sum_{a in A, b in B} v_a v_b Z[c_b, r_a] Z[c_a, r_b]."""
    k = len(coo)
    F = np.zeros((k, k))
    for i, (ra, ca, va) in enumerate(coo):
        for j, (rb, cb, vb) in enumerate(coo):
            z1 = Z[np.ix_(cb, ra)]             # [beta][alpha]
            z2 = Z[np.ix_(ca, rb)]             # [alpha][beta]
            F[i, j] = 0.5 * np.sum(vb[:, None] * va[None, :] * z1 * z2.T)
    return F


def quadratic_from_w(w, coo):
    """Eq. q_harmonic without the bias: y_A = 1/2 w^T E_A w; w is [nmaps][k]."""
    w = np.atleast_2d(w)
    return np.stack([0.5 * np.sum(v[None, :] * w[:, r] * w[:, c], axis=1) for r, c, v in coo], axis=1)


def bias_from_z(Z, Lam, coo):
    """b_A = 1/2 tr[E_A (Z - Z Lambda Z)] = 1/2 sum_a v_a X[c_a, r_a]."""
    ZL = Z @ Lam
    out = np.zeros(len(coo))
    for i, (r, c, v) in enumerate(coo):
        zlz = np.sum(ZL[c, :] * Z[:, r].T, axis=1)      # (Z Lambda Z)[c_a, r_a]
        out[i] = 0.5 * np.sum(v * (Z[c, r] - zlz))
    return out


def qml_harmonic(problem, spectra, lo, hi, maps=None, C=None):
    """Fisher, raw y, bias and C_hat = F^-1 (y - b) (Eq. qml_estimate) through Z."""
    Z, Y, modes, fac = projected_inverse(problem, C)
    coo = coo_derivatives(problem, modes, spectra, lo, hi)
    F = fisher_from_z(Z, coo)
    Lam = cv.mode_covariance(modes, problem.cl, problem.bl, problem.pl)
    b = bias_from_z(Z, Lam, coo)
    out = {"F": F, "bias": b, "Z": Z, "modes": modes}
    if maps is not None:
        w = (Y.T @ sla.cho_solve(fac, np.atleast_2d(maps).T)).T
        y = quadratic_from_w(w, coo)
        out["y"] = y
        out["chat"] = deconvolve(F, y - b[None, :])
    return out


def deconvolve(F, q):
    """C_hat = F^-1 q by a Cholesky solve of F (Eqs. qml_estimate, deconvolved); q is [nmaps][k]."""
    fac = sla.cho_factor(F, lower=True)
    return sla.cho_solve(fac, np.atleast_2d(q).T).T


def inverse_sqrt(F, cutoff=1e-12):
    """F^-1/2 = U Xi^-1/2 U^T from the eigendecomposition F = U Xi U^T, with eigenvalues below
    cutoff times the largest set to zero (Eq. decorrelated and the regularisation beside it)."""
    xi, U = np.linalg.eigh(np.asarray(F, dtype=np.float64))
    keep = xi > cutoff * xi.max()
    w = np.zeros_like(xi)
    w[keep] = 1.0 / np.sqrt(xi[keep])
    return (U * w[None, :]) @ U.T


def decorrelate(F, q, cutoff=1e-12):
    """C_hat^decorr = F^-1/2 q for each row of q (Eq. decorrelated)."""
    return (inverse_sqrt(F, cutoff) @ np.atleast_2d(q).T).T


def bin_matrix(lmin, lmax, lo, hi):
    """P_Sigma [n_b][n_l]: 1 where l lies in bin b (binning identity of the validation section)."""
    nl = lmax - lmin + 1
    P = np.zeros((len(lo), nl))
    for b, (a, c) in enumerate(zip(lo, hi)):
        P[b, a - lmin:c - lmin + 1] = 1.0
    return P


def band_fiducial(cl, spectra, lo, hi, chat, fields):
    """Fiducial of the next iteration of iterative QML (the paper describes the iteration as
    re-entering the pipeline with the previous estimates in place of the fiducial, Sects. 2.2 and
    6; the rules below are readings): every estimated band C_hat[s, b] replaces the fiducial of
    spectrum s as a flat band over the multipoles of bin b; then, at every multipole, the spectrum
    matrix over the problem's harmonic fields (T; E, B; or T, E, B) is replaced by its nearest
    positive semi-definite matrix (negative eigenvalues set to zero), so that the next covariance
    stays positive definite.  cl: [6][lmax + 1] in TT, EE, BB, TE, TB, EB order."""
    new = np.array(cl, dtype=np.float64, copy=True)
    for k, (s, a, b) in enumerate(parameters(spectra, lo, hi)):
        new[SPECS.index(s), a:b + 1] = chat[k]
    harm = [f for f in ("T", "E", "B") if (f == "T" and "T" in fields) or (f != "T" and "Q" in fields)]
    idx = {("T", "T"): 0, ("E", "E"): 1, ("B", "B"): 2, ("T", "E"): 3, ("T", "B"): 4, ("E", "B"): 5}
    for l in range(new.shape[1]):
        M = np.zeros((len(harm), len(harm)))
        for i, a in enumerate(harm):
            for j, b in enumerate(harm):
                key = (a, b) if (a, b) in idx else (b, a)
                M[i, j] = new[idx[key], l]
        xi, U = np.linalg.eigh(M)
        if xi.min() >= 0.0:
            continue
        P = (U * np.maximum(xi, 0.0)[None, :]) @ U.T
        for i, a in enumerate(harm):
            for j, b in enumerate(harm):
                if j >= i:
                    key = (a, b) if (a, b) in idx else (b, a)
                    new[idx[key], l] = P[i, j]
    return new


def iterate(problem, spectra, lo, hi, data, max_iter=20, tol=1e-6):
    """Iterative QML for one map: C_hat^(i) = F(C^(i))^-1 (y - b)(C^(i)) with C^(0) the problem's
    fiducial and C^(i+1) = band_fiducial(C_hat^(i)); stops when no band moves by more than tol of
    its Fisher error sqrt((F^-1)_bb) between two iterations.  Returns (C_hat, F, iterations)."""
    p = problem.__class__(**{**problem.__dict__})
    p.cl = np.array(problem.cl, dtype=np.float64, copy=True)
    prev = None
    for it in range(1, max_iter + 1):
        r = qml_harmonic(p, spectra, lo, hi, np.atleast_2d(data))
        chat = r["chat"][0]
        if prev is not None:
            sig = np.sqrt(np.diag(np.linalg.inv(r["F"])))
            if np.max(np.abs(chat - prev) / sig) < tol:
                return chat, r["F"], it
        prev = chat
        p.cl = band_fiducial(p.cl, spectra, lo, hi, chat, problem.fields)
    return chat, r["F"], max_iter
