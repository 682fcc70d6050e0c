"""Pins of the oracle's decorrelated normalisation (Eq. decorrelated, Sect. 2.5): the covariance of
F^-1/2 q is the identity when Cov(q) = F, (F^-1/2)^2 = F^-1, F^-1/2 commutes with F, the
regularisation removes exactly the directions below the cutoff, and the QML pipeline's deconvolved
and decorrelated estimates differ by the window F^1/2 (<C^decorr> = F^1/2 C)."""
import numpy as np

from oracle import qml

from oracle_cases import tiny_healpix


def _spd(k, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    xi = np.logspace(0, np.log10(cond), k)
    return (Q * xi[None, :]) @ Q.T


def test_inverse_sqrt_algebra():
    F = _spd(40, 5)
    R = qml.inverse_sqrt(F)
    np.testing.assert_allclose(R, R.T, atol=1e-12)
    np.testing.assert_allclose(R @ F @ R, np.eye(40), atol=1e-10)          # Cov(F^-1/2 q) = I
    np.testing.assert_allclose(R @ R, np.linalg.inv(F), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(R @ F, F @ R, atol=1e-9)


def test_inverse_sqrt_of_a_diagonal_and_the_cutoff():
    F = np.diag([4.0, 1.0, 0.25, 1e-14])
    R = qml.inverse_sqrt(F)
    np.testing.assert_allclose(R, np.diag([0.5, 1.0, 2.0, 0.0]), atol=1e-15)
    # rank-deficient F: F^-1/2 F F^-1/2 is the projector on the kept eigenvectors
    rng = np.random.default_rng(9)
    B = rng.standard_normal((12, 8))
    F = B @ B.T                                     # rank 8
    R = qml.inverse_sqrt(F)
    P = R @ F @ R
    np.testing.assert_allclose(P @ P, P, atol=1e-9)
    assert abs(np.trace(P) - 8.0) < 1e-9


def test_decorrelated_estimates_of_a_qml_run():
    """<q> = F C for the fiducial C, so <F^-1/2 q> = F^1/2 C: the decorrelated estimate of the
    expected q is the window F^1/2 applied to the deconvolved one."""
    p = tiny_healpix("QU", nside=2, lmax=5, cut=0.25, lowrank=2)
    spectra, lo, hi = ("EE", "BB"), [2, 4], [3, 5]
    F = qml.fisher_dense(p, spectra, lo, hi)
    C_true = np.array([1.3, 0.7, 0.4, 0.9])
    q = F @ C_true
    dec = qml.decorrelate(F, q)[0]
    xi, U = np.linalg.eigh(F)
    half = (U * np.sqrt(xi)[None, :]) @ U.T
    np.testing.assert_allclose(dec, half @ C_true, rtol=1e-9)
    np.testing.assert_allclose(qml.deconvolve(F, q)[0], C_true, rtol=1e-9)
