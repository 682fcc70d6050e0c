"""More pins of the oracle against identities that do not use its own assembly:

* the projected inverse by two routes: Z = Y^T C^-1 Y directly and the stable SMW form
  M (I + Lambda M)^-1 with M = Y^T N^-1 Y (Eq. smw_stable), and the data weighting
  Y^T C^-1 d = (I + M Lambda)^-1 Y^T N^-1 d (Eq. smw_stable_data);
* E/B separation: on an exact-quadrature full-sky grid, the quadrature projection of the
  pixel-pair covariance of a pure-E sky onto the harmonic basis has no B power and returns
  C^EE_l W_l on the E modes;
* seeded Monte Carlo: E[chi^2] = n for maps drawn from C;
* the scan model: E[-2 ln L(theta)] = tr[C(theta)^-1 C_true] + ln|C(theta)| has, at the true
  parameters, the Hessian 2 F_theta (twice the Fisher matrix in the amplitude parameters), checked
  by central finite differences of the trace and log-determinant."""
import numpy as np
import scipy.linalg as sla

from oracle import covariance as cv
from oracle import healpix, likelihood, qml
from paper_2605_21149_amd import inputs as I

from oracle_cases import gl_problem, tiny_healpix


def test_projected_inverse_two_routes_and_stable_data_weighting():
    p = tiny_healpix("TQU", nside=2, lmax=5, cut=0.3, lowrank=2)
    Z, Y, modes, fac = qml.projected_inverse(p)
    N = p.noise_matrix()
    Lam = cv.mode_covariance(modes, p.cl, p.bl, p.pl)
    M = Y.T @ np.linalg.solve(N, Y)
    k = M.shape[0]
    Z2 = M @ np.linalg.inv(np.eye(k) + Lam @ M)                       # Eq. smw_stable
    np.testing.assert_allclose(Z2, Z, rtol=0, atol=1e-10 * np.abs(Z).max())
    d = np.random.default_rng(5).standard_normal((p.n, 2))
    w = Y.T @ sla.cho_solve(fac, d)
    w2 = np.linalg.solve(np.eye(k) + M @ Lam, Y.T @ np.linalg.solve(N, d))   # Eq. smw_stable_data
    np.testing.assert_allclose(w2, w, rtol=0, atol=1e-10 * np.abs(w).max())


def test_pure_e_sky_has_no_b_power_on_an_exact_quadrature_grid():
    lmax = 6
    p = gl_problem("QU", lmax, 1.0)
    cl = np.zeros_like(p.cl)
    cl[1, 2:] = np.linspace(1.0, 0.4, lmax - 1)                       # EE only
    th, ph = healpix.active_directions(0, None, p.theta, p.phi)
    S = cv.signal_pairs(th, ph, "QU", cl, p.bl, p.pl, p.lmin, p.lmax)
    Y, modes = cv.harmonic_basis(th, ph, "QU", p.lmin, p.lmax)
    w = np.tile(p.extra["weights"], 2)
    A = (Y * w[:, None]).T @ S @ (Y * w[:, None])                      # projected mode covariance
    Wl = cv.window(p.bl, p.pl)
    for j, (f, l, m, cs) in enumerate(modes):
        target = cl[1, l] * Wl[l] if f == "E" else 0.0
        assert abs(A[j, j] - target) < 1e-11 * cl[1].max()
    iB = [j for j, mo in enumerate(modes) if mo[0] == "B"]
    assert np.abs(A[np.ix_(iB, iB)]).max() < 1e-11 * cl[1].max()
    assert np.abs(A - np.diag(np.diag(A))).max() < 1e-11 * cl[1].max()


def test_monte_carlo_mean_chi2_equals_n():
    p = tiny_healpix("QU", nside=2, lmax=5, cut=0.25, lowrank=2)
    C = cv.total_covariance(p)
    nsim = 4000
    d = (np.linalg.cholesky(C) @ np.random.default_rng(906).standard_normal((p.n, nsim))).T
    chi2, _ = likelihood.chi2_logdet(C, d)
    assert abs(chi2.mean() - p.n) < 4.0 * np.sqrt(2.0 * p.n / nsim)


def test_scan_model_hessian_of_expected_likelihood_is_twice_the_fisher():
    p = tiny_healpix("QU", nside=2, lmax=6, cut=0.25)
    p.cl = p.cl.copy()
    p.cl[5] = 0.0
    theta0 = np.full(7, 1.0)
    base = I.scan_spectra(theta0[None], p.cl)[0]

    def cov(theta):
        q = p.__class__(**{**p.__dict__})
        q.cl = I.scan_spectra(np.asarray(theta)[None], base)[0]
        return cv.total_covariance(q)

    C_true = cov(theta0)
    active = [0, 1, 6]                                                   # parameters that move l <= 6

    def f(theta):
        C = cov(theta)
        fac = sla.cho_factor(C, lower=True)
        return np.trace(sla.cho_solve(fac, C_true)) + 2.0 * np.sum(np.log(np.diag(fac[0])))

    h = 1e-3
    H = np.zeros((3, 3))
    for a, i in enumerate(active):
        for b, j in enumerate(active):
            def at(si, sj):
                t = theta0.copy()
                t[i] += si * h
                t[j] += sj * h
                return f(t)
            H[a, b] = (at(1, 1) - at(1, -1) - at(-1, 1) + at(-1, -1)) / (4 * h * h)
    fac = sla.cho_factor(C_true, lower=True)
    dC = []
    for i in active:                                                    # C is linear in theta
        t = theta0.copy()
        t[i] += 1.0
        dC.append(sla.cho_solve(fac, cov(t) - C_true))
    F = np.array([[0.5 * np.sum(x * y.T) for y in dC] for x in dC])
    np.testing.assert_allclose(H, 2.0 * F, rtol=2e-5, atol=1e-8 * np.abs(F).max())
