"""GPU parity of the headline TQU N_side 16 workload (n = 5952, 6 spectra x 12 bins, dense noise)
against the oracle, in the launch configurations bench.py times:

* the FP64 likelihood batch (8 points x 64 maps) after the autotuner has picked its launch shape
  on a fresh table, exactly as the bench's warmup does: every map of three sampled points against
  the oracle's Cholesky likelihood at 1e-10 relative (Eq. pixel_likelihood);
* the mixed-precision likelihood (FP32 and split-BF16x3 with FP64 refinement) against the oracle:
  |d(-2 ln L)| <= 1e-3 absolute, chi^2 within 1e-5;
* the mixed-precision Fisher matrix and QML estimates against the oracle's QML of the same map:
  F within 1e-6 (relative Frobenius), y, noise bias and C_hat within 1e-5 Fisher errors;
* the harmonic-basis (SMW) likelihood with the TEB window l 2..29 against the oracle's SMW
  likelihood (Eqs. smw, logdet) at one point.

The oracle side runs on the host (about 15 s per covariance and factorisation of n = 5952)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import covariance as cv, likelihood, qml, smw  # noqa: E402
from paper_2605_21149_amd import inputs as I  # noqa: E402
from gpu_common import metric_chat, metric_vec_fisher, say, to_np  # noqa: E402

pytestmark = pytest.mark.gpu
SAMPLED = (0, 3, 7)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    from paper_2605_21149_amd import cf
    cf.lib()
    assert torch.cuda.is_available(), "GPU tests selected but torch sees no GPU"


def _cf():
    from paper_2605_21149_amd import cf
    return cf


@pytest.fixture(scope="module")
def workload():
    """The bench's inputs: problem, 64 white maps of rms 3 uK (seed 403), 8 scan points (seed 401)."""
    p = I.tqu_problem_nside16(dense_noise=True)
    maps = I.white_maps(p.n, 64, 403, rms=3.0)
    clp = I.scan_spectra(I.scan_points(8, seed=401), p.cl)[:, None]
    return p, maps, clp


@pytest.fixture(scope="module")
def oracle_points(workload):
    """Oracle -2 ln L (64 maps) and ln|C| at the sampled points."""
    p, maps, clp = workload
    out = {}
    for i in SAMPLED:
        say(f"oracle likelihood at point {i} ...")
        m2, chi2, ld = likelihood.minus2lnL(p, maps, cl=clp[i, 0])
        out[i] = (m2, chi2, ld)
    return out


def _run_scan(p, maps, clp, precision, autotune):
    import torch
    cf = _cf()
    pk = cf.pack_problem(p, device=True)
    d_maps = torch.as_tensor(maps).cuda()
    d_cl = torch.as_tensor(np.ascontiguousarray(clp)).cuda()
    r = cf.loglike_batch([p], d_cl, [d_maps], precision=precision, device=True, packed=[pk],
                         autotune=autotune)
    return {k: to_np(v) for k, v in r.items()}


@pytest.mark.timeout(900)
def test_fp64_scan_autotuned_shape_matches_oracle(workload, oracle_points, tmp_path, monkeypatch):
    """The likelihood batch of the bench: the first call tunes its launch shape into a fresh table
    (points per batch, panel width, GEMM tile), the second runs the scan in that shape; every one of
    the 64 maps at three sampled points against the oracle at 1e-10 relative."""
    p, maps, clp = workload
    cache = tmp_path / "autotune.txt"
    monkeypatch.setenv("CF_TUNE_CACHE", str(cache))
    say("fp64 scan, autotune on a fresh table ...")
    first = _run_scan(p, maps, clp, _cf().CF_FP64, autotune=True)
    lines = [l.strip() for l in open(cache) if l.startswith("scan ")]
    assert lines, "the autotuner wrote no entry"
    say("  tuned:", lines[-1])
    got = _run_scan(p, maps, clp, _cf().CF_FP64, autotune=True)
    for i in SAMPLED:
        m2, _, ld = oracle_points[i]
        for res, name in ((first, "tuning call"), (got, "tuned call")):
            e = float(np.max(np.abs(res["m2lnL"][i, 0] - m2) / np.abs(m2)))
            el = abs(res["logdet"][i, 0] - ld) / abs(ld)
            say(f"  point {i} {name}: max rel -2lnL {e:.2e}, ln|C| {el:.2e}")
            assert e < 1e-10
            assert el < 1e-10


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec_name", ["CF_MIXED_FP32", "CF_MIXED_BF16X3"])
def test_mixed_scan_matches_oracle(workload, oracle_points, prec_name):
    """Mixed-precision likelihood of the bench batch against the oracle: |d(-2 ln L)| <= 1e-3 and
    |d chi^2| <= 1e-5 at the sampled points (every map)."""
    p, maps, clp = workload
    cf = _cf()
    say(f"mixed scan {prec_name} ...")
    got = _run_scan(p, maps, clp, getattr(cf, prec_name), autotune=False)
    for i in SAMPLED:
        m2, chi2, ld = oracle_points[i]
        dm = float(np.max(np.abs(got["m2lnL"][i, 0] - m2)))
        dx = float(np.max(np.abs(got["chi2"][i, 0] - chi2)))
        say(f"  point {i}: |d(-2lnL)| {dm:.2e}, |d chi2| {dx:.2e}, |d ln|C|| {abs(got['logdet'][i, 0] - ld):.2e}")
        assert dm <= 1e-3
        assert dx <= 1e-5


@pytest.fixture(scope="module")
def oracle_qml(workload):
    p = workload[0]
    bins = I.uniform_bins(2, 47, 4, I.SPEC_NAMES)
    maps = I.white_maps(p.n, 1, 202, rms=3.0)
    say("oracle QML (n = 5952, 6900 modes) ...")
    C = cv.total_covariance(p)
    ref = qml.qml_harmonic(p, bins.spectra, bins.lo, bins.hi, maps, C)
    return bins, maps, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec_name", ["CF_FP64", "CF_MIXED_FP32", "CF_MIXED_BF16X3"])
def test_fisher_qml_matches_oracle(workload, oracle_qml, prec_name):
    """F, y, noise bias and C_hat of the bench's Fisher + QML against the oracle: FP64 at 1e-10
    (Fisher-normalised entries, Fisher-error units); mixed paths F within 1e-6 relative Frobenius
    and y, bias, C_hat within 1e-5 Fisher errors."""
    cf = _cf()
    p = workload[0]
    bins, maps, ref = oracle_qml
    prec = getattr(cf, prec_name)
    say(f"fisher+qml {prec_name} ...")
    got = {k: to_np(v) for k, v in cf.qml(p, bins, maps, precision=prec, device=True).items()}
    F = ref["F"]
    d = np.sqrt(np.diag(F))
    m = {"F_norm": float(np.max(np.abs(got["F"] - F) / np.outer(d, d))),
         "F_relfro": float(np.linalg.norm(got["F"] - F) / np.linalg.norm(F)),
         "y": metric_vec_fisher(got["y"], ref["y"], F),
         "bias": metric_vec_fisher(got["bias"], ref["bias"], F),
         "chat": metric_chat(got["chat"], ref["chat"], F)}
    say("  metrics", m)
    if prec == cf.CF_FP64:
        assert all(v < 1e-10 for v in m.values()), m
    else:
        assert m["F_relfro"] <= 1e-6, m
        assert max(m["y"], m["bias"], m["chat"]) < 1e-5, m


@pytest.mark.timeout(900)
def test_smw_tqu_window_matches_oracle_smw(workload):
    """The harmonic-basis likelihood of the TQU problem with the TEB window l 2..29 (2688 modes) at
    one scan point against the oracle's SMW likelihood (Eqs. K_kernel, smw, logdet).  Tolerance
    1e-8 relative: the FP64 solves against N_eff (kappa about 1.2e4 at n = 5952) carry relative
    errors up to about n u kappa = 8e-9 by the standard backward-error bound, and the data term's
    difference d^T N_eff^-1 d - |L^-1 b'|^2 (about 2.05e4 - 0.5e4 = 1.55e4 per map here) amplifies
    them by no more than 1.3."""
    import torch
    cf = _cf()
    p, maps, clp = workload
    maps4 = maps[:4]
    pt = clp[3, 0]
    d_maps = torch.as_tensor(maps4).cuda()
    with cf.SMW(p, d_maps, (2, 29), "TEB", device=True) as h:
        got = {k: to_np(v) for k, v in h.loglike(torch.as_tensor(pt[None].copy()).cuda()).items()}
    say("oracle SMW likelihood ...")
    m2, chi2, ld = smw.smw_minus2lnL(p, maps4, pt, 2, 29, "TEB")
    e = float(np.max(np.abs(got["m2lnL"][0] - m2) / np.abs(m2)))
    el = abs(got["logdet"][0] - ld) / abs(ld)
    say(f"  max rel -2lnL {e:.2e}, ln|C| {el:.2e}")
    assert e < 1e-8
    assert el < 1e-8
