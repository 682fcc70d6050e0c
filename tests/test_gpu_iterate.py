"""GPU parity of iterative QML (cf_qml_iterate) against the oracle's iteration (oracle/qml.py
iterate, pinned by the stationarity of the exact pixel likelihood at its fixed point): the same
number of iterations, and C-hat and F at the last fiducial, for a TQU problem with all six spectra
(host and device memory) and a noisy QU problem whose fixed point has the positive semi-definite
projection of the spectra active; a T problem whose fixed point is checked for stationarity of
the oracle's likelihood directly, with the last fiducial returned; and the error paths."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import covariance as cv, likelihood, qml  # noqa: E402
from gpu_common import metric_chat, metric_F, say, to_np  # noqa: E402
from oracle_cases import tiny_healpix  # noqa: E402
from paper_2605_21149_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    from paper_2605_21149_amd import cf
    cf.lib()
    assert torch.cuda.is_available(), "GPU tests selected but torch sees no GPU"


def _cf():
    from paper_2605_21149_amd import cf
    return cf


def _data(p, seed):
    C = cv.total_covariance(p)
    return np.linalg.cholesky(C) @ np.random.default_rng(seed).standard_normal(p.n)


CASES = [  # fields, spectra, noise, low-rank noise modes, map seed; device memory
    ("TQU", I.SPEC_NAMES, 0.5, 2, 81, True),
    ("TQU", I.SPEC_NAMES, 0.5, 2, 81, False),
    ("QU", ("EE", "BB", "EB"), 2.0, 0, 91, True),     # projection active at the fixed point
]


@pytest.mark.parametrize("fields,spectra,noise,lowrank,seed,device", CASES)
def test_iterate_against_oracle(fields, spectra, noise, lowrank, seed, device):
    cf = _cf()
    p = tiny_healpix(fields, nside=4, lmax=9, cut=0.25, noise=noise, lowrank=lowrank)
    lo = np.array([2, 4, 6, 8]); hi = lo + 1
    d = _data(p, seed)
    ref_c, ref_F, ref_it = qml.iterate(p, spectra, lo, hi, d, max_iter=80, tol=1e-8)
    bins = I.Bins(lo.astype(np.int32), hi.astype(np.int32), tuple(spectra))
    say("iterate", fields, p.n, "device", device, "oracle iterations", ref_it)
    got = cf.qml_iterate(p, bins, d, max_iter=80, tol=1e-8, device=device)
    say("  GPU iterations", got["iterations"])
    assert got["iterations"] == ref_it
    F = ref_F
    mc = metric_chat(to_np(got["chat"]), ref_c, F)
    mf = metric_F(to_np(got["F"]), F)
    say(f"  chat {mc:.2e}  F {mf:.2e}")
    assert mc < 1e-9 and mf < 1e-10


def test_iterate_t_fixed_point_is_stationary_for_the_oracle_likelihood():
    cf = _cf()
    p = tiny_healpix("T", nside=4, lmax=9, cut=0.25)
    lo = np.array([2, 4, 6, 8]); hi = lo + 1
    d = _data(p, 71)
    bins = I.Bins(lo.astype(np.int32), hi.astype(np.int32), ("TT",))
    got = cf.qml_iterate(p, bins, d, max_iter=60, tol=1e-10, device=True)
    chat, F, cl = to_np(got["chat"]), to_np(got["F"]), got["cl"]
    say("iterate t: iterations", got["iterations"], "chat", chat)
    np.testing.assert_allclose(cl, qml.band_fiducial(p.cl, ("TT",), lo, hi, chat, p.fields), rtol=1e-9, atol=0)
    sig = np.sqrt(np.diag(np.linalg.inv(F)))
    for b in range(len(lo)):
        h = 1e-3 * sig[b]
        f = []
        for sgn in (1, -1):
            c = cl.copy()
            c[0, lo[b]:hi[b] + 1] += sgn * h
            f.append(likelihood.minus2lnL(p, d, cl=c)[0][0])
        g = (f[0] - f[1]) / (2 * h) * sig[b]
        say(f"  band {b}: gradient x sigma {g:.2e}")
        assert abs(g) < 1e-5


def test_iterate_errors():
    cf = _cf()
    p = tiny_healpix("T", nside=2, lmax=6, cut=0.3)
    lo = np.array([2, 4]); hi = np.array([3, 6])
    bins = I.Bins(lo.astype(np.int32), hi.astype(np.int32), ("TT",))
    d = _data(p, 5)
    with pytest.raises(cf.CFError) as e:
        cf.qml_iterate(p, bins, d, max_iter=1, tol=1e-6, device=True)   # no second iterate to compare
    assert e.value.status == cf.CF_ENOCONV
    with pytest.raises(cf.CFError) as e:
        cf.qml_iterate(p, bins, d, max_iter=5, tol=0.0, device=True)
    assert e.value.status == cf.CF_EINVAL
