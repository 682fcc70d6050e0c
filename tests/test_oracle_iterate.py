"""Pins of the oracle's iterative QML (oracle/qml.py: band_fiducial, iterate).

The paper states that the single-step QML estimate is one Newton step towards the maximum of the
pixel likelihood (Eq. pixel_likelihood) and that iterative QML converges to that maximum
(Sects. 2.2 and 2.6).  With bins that cover every multipole of every spectrum of the fields, the
covariance is N + sum_b C_b P_b exactly, so at the fixed point the exact likelihood, computed by
the direct Cholesky route and not by the QML code, must be stationary in the band amplitudes:
checked by central finite differences.  Also: the spectrum projection keeps S positive
semi-definite and leaves a positive semi-definite spectrum unchanged."""
import numpy as np

from oracle import covariance as cv
from oracle import likelihood, qml

from oracle_cases import tiny_healpix


def _data(p, seed):
    C = cv.total_covariance(p)
    return np.linalg.cholesky(C) @ np.random.default_rng(seed).standard_normal(p.n)


def test_iterative_qml_converges_to_a_stationary_point_of_the_pixel_likelihood():
    p = tiny_healpix("T", nside=4, lmax=9, cut=0.25)
    lo = np.array([2, 4, 6, 8]); hi = lo + 1
    d = _data(p, 71)
    chat, F, it = qml.iterate(p, ("TT",), lo, hi, d, max_iter=60, tol=1e-10)
    assert it < 60
    assert np.all(chat > 0)                                   # the projection stays inactive
    cl = qml.band_fiducial(p.cl, ("TT",), lo, hi, chat, p.fields)
    sig = np.sqrt(np.diag(np.linalg.inv(F)))
    for b in range(len(lo)):
        h = 1e-3 * sig[b]
        f = []
        for sgn in (1, -1):
            c = cl.copy()
            c[0, lo[b]:hi[b] + 1] += sgn * h
            f.append(likelihood.minus2lnL(p, d, cl=c)[0][0])
        g = (f[0] - f[1]) / (2 * h)
        assert abs(g) * sig[b] < 1e-5, (b, g * sig[b])
    # one step from a fiducial far off moves -2 ln L downhill, the fixed point is lower still
    start = likelihood.minus2lnL(p, d)[0][0]
    assert likelihood.minus2lnL(p, d, cl=cl)[0][0] < start


def test_first_iteration_is_the_single_step_estimate():
    p = tiny_healpix("QU", nside=2, lmax=6, cut=0.3)
    lo = np.array([2, 4]); hi = np.array([3, 6])
    spectra = ("EE", "BB", "EB")
    d = _data(p, 72)
    one = qml.qml_harmonic(p, spectra, lo, hi, d[None, :])["chat"][0]
    chat, _, it = qml.iterate(p, spectra, lo, hi, d, max_iter=1)
    assert it == 1
    np.testing.assert_array_equal(chat, one)


def test_band_projection_is_psd_and_idempotent_on_psd_spectra():
    p = tiny_healpix("TQU", nside=2, lmax=6, cut=0.3)
    lo = np.array([2, 5]); hi = np.array([4, 6])
    spectra = ("TT", "EE", "BB", "TE", "TB", "EB")
    rng = np.random.default_rng(73)
    chat = rng.normal(0.0, 1.0, 12)                          # arbitrary, indefinite bands
    new = qml.band_fiducial(p.cl, spectra, lo, hi, chat, p.fields)
    for l in range(2, 7):
        M = np.array([[new[0, l], new[3, l], new[4, l]], [new[3, l], new[1, l], new[5, l]],
                      [new[4, l], new[5, l], new[2, l]]])
        assert np.linalg.eigvalsh(M).min() > -1e-12 * max(1.0, np.abs(M).max())
    again = qml.band_fiducial(new, (), lo[:0], hi[:0], np.zeros(0), p.fields)
    np.testing.assert_allclose(again, new, rtol=0, atol=1e-12 * np.abs(new).max())


def test_band_projection_for_t_and_qu_fields():
    """T: a negative TT band becomes zero and a positive one is kept.  QU: the 2 x 2 (EE, EB; EB, BB)
    matrix of an indefinite band becomes its positive part (closed form of the 2 x 2 case) and TT,
    TE, TB rows stay untouched."""
    lo = np.array([2, 4]); hi = np.array([3, 6])
    p = tiny_healpix("T", nside=2, lmax=6, cut=0.3)
    new = qml.band_fiducial(p.cl, ("TT",), lo, hi, np.array([-0.3, 0.7]), p.fields)
    assert np.all(new[0, 2:4] == 0.0) and np.all(new[0, 4:7] == 0.7)
    p = tiny_healpix("QU", nside=2, lmax=6, cut=0.3)
    chat = np.array([1.0, 0.5, 0.25, 0.2, 0.9, 0.1])           # EE, BB, EB bands (2 bins each)
    new = qml.band_fiducial(p.cl, ("EE", "BB", "EB"), lo, hi, chat, p.fields)
    M = np.array([[1.0, 0.9], [0.9, 0.25]])                     # bin 0: EE 1, BB 0.25, EB 0.9
    xi, U = np.linalg.eigh(M)
    P = (U * np.maximum(xi, 0)[None, :]) @ U.T
    for l in (2, 3):
        np.testing.assert_allclose([new[1, l], new[2, l], new[5, l]], [P[0, 0], P[1, 1], P[0, 1]],
                                   rtol=0, atol=1e-14)
    for l in (4, 5, 6):                                          # bin 1 is positive definite: kept
        np.testing.assert_array_equal([new[1, l], new[2, l], new[5, l]], [0.5, 0.2, 0.1])
    np.testing.assert_array_equal(new[[0, 3, 4]], p.cl[[0, 3, 4]])


def test_band_projection_tqu_indefinite_band_closed_form():
    """A TEB band built as U diag(2, 1, -1/2) U^T with the rational orthonormal basis
    u1 = (2, 1, -2)/3, u2 = (2, -2, 1)/3, u3 = (1, 2, 2)/3: its nearest positive semi-definite
    matrix is 2 u1 u1^T + u2 u2^T, i.e. the band plus u3 u3^T / 2, written entry by entry below in
    ninths.  Every TT, EE, BB, TE, TB and EB entry of the projected band is checked one by one, the
    other bin (positive definite) is left as given."""
    p = tiny_healpix("TQU", nside=2, lmax=6, cut=0.3)
    lo = np.array([2, 5]); hi = np.array([4, 6])
    spectra = ("TT", "EE", "BB", "TE", "TB", "EB")
    # M = 2 u1 u1^T + u2 u2^T - u3 u3^T / 2, in ninths: u_i u_i^T = (outer of the integer vectors) / 9
    # u1 u1^T*9 = [[4,2,-4],[2,1,-2],[-4,-2,4]];  u2 u2^T*9 = [[4,-4,2],[-4,4,-2],[2,-2,1]]
    # u3 u3^T*9 = [[1,2,2],[2,4,4],[2,4,4]]
    # M*9 = [[8+4-0.5, 4-4-1, -8+2-1], [., 2+4-2, -4-2-2], [., ., 8+1-2]] = [[11.5,-1,-7],[-1,4,-8],[-7,-8,7]]
    TT, EE, BB, TE, TB, EB = 11.5 / 9, 4 / 9, 7 / 9, -1 / 9, -7 / 9, -8 / 9
    # P*9 = [[12,0,-6],[0,6,-6],[-6,-6,9]]
    P = {"TT": 12 / 9, "EE": 6 / 9, "BB": 9 / 9, "TE": 0.0, "TB": -6 / 9, "EB": -6 / 9}
    M = np.array([[TT, TE, TB], [TE, EE, EB], [TB, EB, BB]])
    assert np.allclose(np.sort(np.linalg.eigvalsh(M)), [-0.5, 1.0, 2.0], atol=1e-14)
    good = [3.0, 2.0, 1.0, 0.5, 0.1, 0.2]                      # bin 1: positive definite
    chat = np.array([v for pair in zip([TT, EE, BB, TE, TB, EB], good) for v in pair])
    new = qml.band_fiducial(p.cl, spectra, lo, hi, chat, p.fields)
    row = {"TT": 0, "EE": 1, "BB": 2, "TE": 3, "TB": 4, "EB": 5}
    for name, val in P.items():
        for l in (2, 3, 4):
            assert abs(new[row[name], l] - val) <= 1e-14, (name, l, new[row[name], l], val)
    for k, name in enumerate(spectra):
        for l in (5, 6):
            assert new[row[name], l] == good[k], (name, l)
