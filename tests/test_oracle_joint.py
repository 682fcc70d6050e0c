"""Pins of the oracle's joint two-map estimator (Eq. C_joint: one sky seen by two data sets, the
standard QML applied to the stacked 2n-dimensional system):
* two data sets with the same noise and no shared noise are, after the rotation u = (d1 + d2)/sqrt 2,
  v = (d1 - d2)/sqrt 2, a signal-free v and a u of signal 2S and noise N: the joint estimator equals
  the single-map estimator of the mean map (d1 + d2)/2 with noise N/2 (F, y, bias and C_hat of
  independent oracle functions);
* with the inter-map signal switched off (s12 = 0) and no shared noise the system is block
  diagonal: F, y and bias are the sums of the two single-map estimators';
* with noise shared between the data sets (N12 != 0) and unequal noises, the mean of C_hat over
  seeded draws d = (s + n1, s + n2), s from S = sum_B C_B P_B, matches C_B within 5 Monte Carlo
  standard errors, while the same draws analysed as if N12 were zero miss it."""
import copy

import numpy as np

from oracle import covariance as cv
from oracle import qml

from oracle_cases import tiny_healpix

SPECTRA, LO, HI = ("EE", "BB", "EB"), [2, 4], [3, 5]


def _problem():
    return tiny_healpix("QU", nside=2, lmax=5, cut=0.25, lowrank=2)


def test_joint_of_equal_noise_splits_is_the_mean_map_estimator():
    p = _problem()
    rng = np.random.default_rng(11)
    d1, d2 = rng.standard_normal((2, p.n)), rng.standard_normal((2, p.n))
    got = qml.joint_dense(p, p, SPECTRA, LO, HI, d1, d2)
    half = copy.copy(p)
    half.noise_diag = p.noise_diag / 2.0
    half.noise_U = p.noise_U / np.sqrt(2.0)
    m = 0.5 * (d1 + d2)
    F = qml.fisher_dense(half, SPECTRA, LO, HI)
    y = qml.quadratic_dense(half, SPECTRA, LO, HI, m)
    b = qml.bias_dense(half, SPECTRA, LO, HI)
    np.testing.assert_allclose(got["F"], F, rtol=1e-9)
    np.testing.assert_allclose(got["y"], y, rtol=1e-9, atol=1e-12 * np.abs(y).max())
    np.testing.assert_allclose(got["bias"], b, rtol=1e-9)
    np.testing.assert_allclose(got["chat"], qml.deconvolve(F, y - b[None, :]), rtol=1e-8,
                               atol=1e-12 * np.abs(got["chat"]).max())


def test_joint_with_decoupled_skies_is_the_sum_of_two_auto_estimators():
    p1 = _problem()
    p2 = copy.copy(p1)
    rng = np.random.default_rng(5)
    p2.noise_diag = p1.noise_diag * rng.uniform(0.5, 2.0, p1.n)
    p2.noise_U = None
    d1, d2 = rng.standard_normal((2, p1.n)), rng.standard_normal((2, p1.n))
    got = qml.joint_dense(p1, p2, SPECTRA, LO, HI, d1, d2, s12=0.0)
    for key, f in (("F", lambda p, d: qml.fisher_dense(p, SPECTRA, LO, HI)),
                   ("y", lambda p, d: qml.quadratic_dense(p, SPECTRA, LO, HI, d)),
                   ("bias", lambda p, d: qml.bias_dense(p, SPECTRA, LO, HI))):
        want = f(p1, d1) + f(p2, d2)
        np.testing.assert_allclose(got[key], want, rtol=1e-9, atol=1e-12 * np.abs(want).max())


def test_joint_monte_carlo_mean_is_unbiased_with_shared_noise():
    """Shared noise from a common latent z: n1 = e1 + A z, n2 = e2 + B z with B = A R, so
    N1 = D1 + A A^T, N2 = D2 + B B^T and N12 = A B^T (not symmetric: a transposed block would
    show).  A A^T = 0.5 (P_EE,1 + P_EE,2 + P_BB,1 + P_BB,2), so the shared noise lies in the bins'
    modes and ignoring it biases the estimate."""
    p1 = _problem()
    p2 = copy.copy(p1)
    rng = np.random.default_rng(907)
    n = p1.n
    p2.noise_diag = p1.noise_diag * rng.uniform(0.5, 2.0, n)
    pars = qml.parameters(SPECTRA, LO, HI)
    P = [qml.derivative_dense(p1, *p) for p in pars]
    w, V = np.linalg.eigh(0.5 * (P[0] + P[1] + P[2] + P[3]))
    keep = w > 1e-10 * w.max()
    A = V[:, keep] * np.sqrt(w[keep])
    m = A.shape[1]
    B = A @ (0.8 * np.eye(m) + 0.3 * rng.standard_normal((m, m)))
    p1.noise_U, p2.noise_U = A, B
    N12 = A @ B.T
    C_true = np.array([1.0, 0.6, 0.4, 0.7, 0.02, 0.01])
    S = sum(c * Pb for c, Pb in zip(C_true, P))
    M = 4000
    s = np.linalg.cholesky(S + 1e-12 * np.eye(n)) @ rng.standard_normal((n, M))
    z = rng.standard_normal((m, M))
    n1 = np.sqrt(p1.noise_diag)[:, None] * rng.standard_normal((n, M)) + A @ z
    n2 = np.sqrt(p2.noise_diag)[:, None] * rng.standard_normal((n, M)) + B @ z
    d1, d2 = (s + n1).T, (s + n2).T
    got = qml.joint_dense(p1, p2, SPECTRA, LO, HI, d1, d2, N12=N12)
    mean = got["chat"].mean(axis=0)
    err = got["chat"].std(axis=0, ddof=1) / np.sqrt(M)
    assert np.all(np.abs(mean - C_true) < 5.0 * err)
    # the same draws analysed as if the noise were independent keep the shared noise power
    naive = qml.joint_dense(p1, p2, SPECTRA, LO, HI, d1, d2)
    nmean = naive["chat"].mean(axis=0)
    nerr = naive["chat"].std(axis=0, ddof=1) / np.sqrt(M)
    assert np.any(np.abs(nmean - C_true) > 8.0 * nerr)
