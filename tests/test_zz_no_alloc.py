"""cf_loglike_batch_noalloc (the entry point for callers that cannot allocate) against
cf_loglike_batch through the C ABI: two calls in a row, the second on a smaller input, plus the
mixed-precision path and the rejection of a problem whose workspace exceeds the static array."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import covariance as cv, likelihood  # noqa: E402
from paper_2605_21149_amd import inputs as I  # noqa: E402
from gpu_common import say, to_np  # noqa: E402
from oracle_cases import tiny_healpix  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    from paper_2605_21149_amd import cf
    cf.lib()
    assert torch.cuda.is_available(), "GPU tests selected but torch sees no GPU"


def _cf():
    from paper_2605_21149_amd import cf
    return cf


def _both(problems, clp, maps, device, precision=0):
    cf = _cf()
    pks = [cf.pack_problem(p, device=device) for p in problems]
    ref = cf.loglike_batch(problems, clp, maps, precision=precision, device=device, packed=pks)
    got = cf.loglike_batch(problems, clp, maps, precision=precision, device=device, packed=pks, noalloc=True)
    return {k: to_np(v) for k, v in ref.items()}, {k: to_np(v) for k, v in got.items()}


def test_noalloc_matches_loglike_batch_two_calls_second_smaller():
    import torch
    # call 1: the QU N_side 8 scan problem (n = 1088), 64 maps, 12 points, device memory (batches of 4)
    p = I.qu_scan_problem(8)
    maps = I.white_maps(p.n, 64, 402, rms=3.0)
    clp = I.scan_spectra(I.scan_points(12, seed=401), p.cl)[:, None]
    say("noalloc call 1: n", p.n, "64 maps, 12 points, device")
    ref, got = _both([p], torch.as_tensor(clp).cuda(), [torch.as_tensor(maps).cuda()], True)
    e = float(np.max(np.abs(got["m2lnL"] - ref["m2lnL"]) / np.abs(ref["m2lnL"])))
    say(f"  max rel -2lnL vs cf_loglike_batch {e:.2e}")
    assert e < TOL
    np.testing.assert_allclose(got["logdet"], ref["logdet"], rtol=TOL)
    np.testing.assert_allclose(got["chi2"], ref["chi2"], rtol=TOL)
    m2o, _, ldo = likelihood.minus2lnL(p, maps[:2], cl=clp[5, 0])
    np.testing.assert_allclose(got["m2lnL"][5, 0, :2], m2o, rtol=TOL)
    # call 2: a smaller tiny QU problem, 3 maps, 5 points, host memory (inputs staged in the array)
    q = tiny_healpix("QU", nside=2, lmax=6, cut=0.2, lowrank=1)
    mq = (np.linalg.cholesky(cv.total_covariance(q)) @ np.random.default_rng(5).standard_normal((q.n, 3))).T
    clq = I.scan_spectra(I.scan_points(5, seed=6), q.cl)[:, None]
    say("noalloc call 2: n", q.n, "3 maps, 5 points, host")
    ref2, got2 = _both([q], clq, [mq], False)
    e2 = float(np.max(np.abs(got2["m2lnL"] - ref2["m2lnL"]) / np.abs(ref2["m2lnL"])))
    say(f"  max rel -2lnL vs cf_loglike_batch {e2:.2e}")
    assert e2 < TOL
    np.testing.assert_allclose(got2["logdet"], ref2["logdet"], rtol=TOL)
    oref, _ = likelihood.scan(q, mq, clq[:, 0])
    np.testing.assert_allclose(got2["m2lnL"][:, 0], oref, rtol=TOL)


def test_noalloc_mixed_and_two_problems():
    """Two uneven problems in one call and the FP32 mixed path on the single-stream factorisation:
    FP64 within 1e-10 of cf_loglike_batch, FP32 within the mixed budget |d(-2 ln L)| <= 1e-3."""
    pa = tiny_healpix("QU", nside=2, lmax=6, cut=0.2, lowrank=1)
    pb = tiny_healpix("QU", nside=4, lmax=9, cut=0.3, lowrank=2)
    rng = np.random.default_rng(9)
    maps = [rng.standard_normal((2, pa.n)), rng.standard_normal((2, pb.n))]
    pts = I.scan_points(7, seed=8)
    clp = np.zeros((7, 2, 6, pb.lmax + 1))
    clp[:, 0, :, :pa.lmax + 1] = I.scan_spectra(pts, pa.cl)
    clp[:, 1] = I.scan_spectra(pts, pb.cl)
    say("noalloc two problems FP64")
    ref, got = _both([pa, pb], clp, maps, False)
    np.testing.assert_allclose(got["m2lnL"], ref["m2lnL"], rtol=TOL)
    say("noalloc FP32 mixed")
    ref32, got32 = _both([pb], clp[:, 1:], maps[1:], False, precision=_cf().CF_MIXED_FP32)
    d = float(np.max(np.abs(got32["m2lnL"] - ref32["m2lnL"])))
    say(f"  max |d(-2lnL)| FP32 noalloc vs FP32 {d:.2e}")
    assert d <= 1e-3


def test_noalloc_rejects_a_problem_beyond_the_array():
    """The TQU N_side 16 problem (n = 5952) needs about 290 MB for one point: CF_EINVAL with the
    sizes in the message, before any launch."""
    cf = _cf()
    p = I.tqu_problem_nside16(dense_noise=False)
    maps = np.zeros((4, p.n))
    clp = I.scan_spectra(I.scan_points(1, seed=1), p.cl)[:, None]
    with pytest.raises(cf.CFError) as e:
        cf.loglike_batch([p], clp, [maps], noalloc=True)
    assert e.value.status == cf.CF_EINVAL and "scratch" in str(e.value), str(e.value)
