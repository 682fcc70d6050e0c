"""Pins of the oracle's harmonic-basis (Sherman-Morrison-Woodbury) likelihood with multipole
switching (Sects. 2.3.2, 2.3.4, 2.6).  The reference each time is the direct pixel likelihood of
the oracle: the covariance from the pixel-pair route, one Cholesky factorisation of C, no harmonic
basis, so that a wrong Lambda, a wrong split between N_eff and the window or a mistake in the
Woodbury or determinant-lemma algebra shows up as a mismatch."""
import numpy as np
import pytest

from oracle import covariance as cv
from oracle import healpix, likelihood, smw

from oracle_cases import random_spectra, tiny_healpix


def _maps(n, nmaps, seed):
    return np.random.default_rng(seed).standard_normal((nmaps, n))


def _compare(p, maps, cl_point, wlo, whi, wfields):
    m2, chi2, ld = smw.smw_minus2lnL(p, maps, cl_point, wlo, whi, wfields)
    full = smw.window_spectra(p, cl_point, wlo, whi, wfields)
    m2d, chi2d, ldd = likelihood.minus2lnL(p, maps, cl=full)
    np.testing.assert_allclose(chi2, chi2d, rtol=1e-9)
    np.testing.assert_allclose(ld, ldd, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(m2, m2d, rtol=1e-9)
    return m2


def test_switched_split_reassembles_the_fiducial_covariance():
    """Eq. C_switched at the fiducial spectra: N_eff + V_inf^T Lambda_inf V_inf = C."""
    p = tiny_healpix("TQU", nside=2, lmax=6, cut=0.3, lowrank=2)
    wlo, whi, wf = 2, 4, "TEB"
    V, modes = smw.window_basis(p, wlo, whi, wf)
    Lam = cv.mode_covariance(modes, p.cl, p.bl, p.pl)
    C = smw.effective_noise(p, wlo, whi, wf) + V.T @ Lam @ V
    C0 = cv.total_covariance(p)
    np.testing.assert_allclose(C, C0, rtol=0, atol=1e-11 * np.abs(C0).max())


def test_smw_likelihood_equals_direct_all_fields_window():
    p = tiny_healpix("TQU", nside=2, lmax=6, cut=0.3, lowrank=2)
    maps = _maps(p.n, 3, 71)
    point = random_spectra(p.lmax, 99)
    m2 = _compare(p, maps, point, 2, 4, "TEB")
    # the point differs from the fiducial inside the window: the likelihood moves
    m2_fid = _compare(p, maps, p.cl, 2, 4, "TEB")
    assert np.all(np.abs(m2 - m2_fid) > 1e-3)


def test_smw_full_window_is_the_plain_identity():
    """Window = the whole signal band and every field: N_eff = N (Eqs. C_factored, smw, logdet)."""
    p = tiny_healpix("QU", nside=2, lmax=5, cut=0.25, lowrank=2)
    assert np.array_equal(smw.effective_noise(p, p.lmin, p.lmax, "EB"), p.noise_matrix())
    _compare(p, _maps(p.n, 2, 72), random_spectra(p.lmax, 98), p.lmin, p.lmax, "EB")


def test_smw_e_only_window_of_a_qu_problem():
    """Only E varies (EB = 0): B stays in N_eff with its fiducial spectrum."""
    p = tiny_healpix("QU", nside=2, lmax=6, cut=0.25)
    p.cl = p.cl.copy()
    p.cl[5] = 0.0
    point = p.cl.copy()
    point[1, 2:6] *= np.array([0.6, 1.4, 0.8, 1.2])
    point[2] *= 7.0          # BB of the point is not in the varied part: ignored
    m2 = _compare(p, _maps(p.n, 2, 73), point, 2, 5, "E")
    m2_ref = likelihood.minus2lnL(p, _maps(p.n, 2, 73), cl=smw.window_spectra(p, point, 2, 5, "E"))[0]
    np.testing.assert_allclose(m2, m2_ref, rtol=1e-9)


def test_window_coupling_a_varied_and_a_fixed_field_is_rejected():
    p = tiny_healpix("TQU", nside=2, lmax=5, cut=0.3)
    assert np.any(p.cl[3, 2:4] != 0)                  # TE couples T and E
    with pytest.raises(ValueError):
        smw.check_window(p, 2, 3, "E")
    with pytest.raises(ValueError):
        smw.check_window(p, 2, 9, "TEB")              # beyond lmax
    smw.check_window(p, 2, 3, "TEB")
