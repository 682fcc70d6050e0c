"""Pins of the oracle's cross-QML (Eq. q_cross and its mode-mixing matrix): with one data set used
twice it reduces to the auto estimator (quadratic form and Fisher matrix of independent oracle
functions); for two noises its expectation over a shared signal carries no noise term,
<q^x> = W^x C exactly (the trace identity evaluated without the estimator's own assembly); W^x is
symmetric positive definite."""
import copy

import numpy as np
import scipy.linalg as sla

from oracle import covariance as cv
from oracle import qml

from oracle_cases import tiny_healpix

SPECTRA, LO, HI = ("EE", "BB", "EB"), [2, 4], [3, 5]


def _pair(seed_noise=5):
    p1 = tiny_healpix("QU", nside=2, lmax=5, cut=0.25, lowrank=2)
    p2 = copy.copy(p1)
    rng = np.random.default_rng(seed_noise)
    p2.noise_diag = p1.noise_diag * rng.uniform(0.5, 2.0, p1.n)
    p2.noise_U = None
    return p1, p2


def test_cross_with_one_data_set_twice_is_the_auto_estimator():
    p1, _ = _pair()
    maps = np.random.default_rng(1).standard_normal((2, p1.n))
    q, W, chat = qml.cross_dense(p1, p1, SPECTRA, LO, HI, maps, maps)
    np.testing.assert_allclose(q, qml.quadratic_dense(p1, SPECTRA, LO, HI, maps), rtol=1e-10)
    np.testing.assert_allclose(W, qml.fisher_dense(p1, SPECTRA, LO, HI), rtol=1e-10)


def test_cross_expectation_has_no_noise_term_and_w_is_spd():
    """<d1 d2^T> = S for independent noises, so <q^x_A> = 1/2 tr[C1^-1 P_A C2^-1 S]; with
    S = sum_B C_B P_B (the model restricted to the bins) this equals sum_B W^x_AB C_B."""
    p1, p2 = _pair()
    pars = qml.parameters(SPECTRA, LO, HI)
    P = [qml.derivative_dense(p1, *p) for p in pars]
    C_true = np.array([1.2, 0.8, 0.5, 0.9, 0.05, -0.03])
    S = sum(c * Pb for c, Pb in zip(C_true, P))
    C1 = cv.total_covariance(p1)
    C2 = cv.total_covariance(p2)
    f1, f2 = sla.cho_factor(C1, lower=True), sla.cho_factor(C2, lower=True)
    expect = np.array([0.5 * np.trace(sla.cho_solve(f1, Pa) @ sla.cho_solve(f2, S)) for Pa in P])
    _, W, _ = qml.cross_dense(p1, p2, SPECTRA, LO, HI, np.zeros((1, p1.n)), np.zeros((1, p1.n)))
    np.testing.assert_allclose(W @ C_true, expect, rtol=1e-10, atol=1e-12 * np.abs(expect).max())
    np.testing.assert_allclose(W, W.T, rtol=1e-10, atol=1e-14 * np.abs(W).max())
    assert np.linalg.eigvalsh(W).min() > 0


def test_cross_monte_carlo_mean_is_unbiased_without_noise_correction():
    """Seeded draws d1 = s + n1, d2 = s + n2 (shared signal from S = sum_B C_B P_B, independent
    noises): the mean of q^x matches W^x C within 5 Monte Carlo standard errors."""
    p1, p2 = _pair(7)
    pars = qml.parameters(SPECTRA, LO, HI)
    P = [qml.derivative_dense(p1, *p) for p in pars]
    C_true = np.array([1.0, 0.6, 0.4, 0.7, 0.02, 0.01])
    S = sum(c * Pb for c, Pb in zip(C_true, P))
    rng = np.random.default_rng(902)
    M = 4000
    Ls = np.linalg.cholesky(S + 1e-12 * np.eye(p1.n))
    L1 = np.linalg.cholesky(p1.noise_matrix())
    L2 = np.linalg.cholesky(p2.noise_matrix())
    s = Ls @ rng.standard_normal((p1.n, M))
    d1 = (s + L1 @ rng.standard_normal((p1.n, M))).T
    d2 = (s + L2 @ rng.standard_normal((p1.n, M))).T
    q, W, _ = qml.cross_dense(p1, p2, SPECTRA, LO, HI, d1, d2)
    mean, err = q.mean(axis=0), q.std(axis=0, ddof=1) / np.sqrt(M)
    assert np.all(np.abs(mean - W @ C_true) < 5.0 * err)
