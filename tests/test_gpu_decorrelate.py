"""GPU parity of the decorrelated normalisation (cf_decorrelate, Eq. decorrelated) against the
oracle's eigendecomposition: conditioned SPD matrices, odd K (the round-robin's idle index), a
rank-deficient F (the eigenvalue cutoff), an F whose upper triangle is garbage (only the lower one
is read), and the Fisher matrix and raw estimates of a QML run."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import qml  # noqa: E402
from gpu_common import say, to_np  # noqa: E402
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


def _spd(k, seed, cond):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    xi = np.logspace(0, np.log10(cond), k)
    return (Q * xi[None, :]) @ Q.T


def _check(F, q, device, tol=1e-10):
    cf = _cf()
    (out, R), rep = cf.decorrelate(F, q, device=device, report=True)
    R_ref = qml.inverse_sqrt(F)
    scale = np.abs(R_ref).max()
    assert np.abs(to_np(R) - R_ref).max() <= tol * scale
    if q is not None:
        ref = qml.decorrelate(F, q)
        assert np.abs(to_np(out) - ref).max() <= tol * np.abs(ref).max()
    say(f"  K={F.shape[0]}: sweeps {rep['ir_iters']}, max |dR|/max|R| {np.abs(to_np(R) - R_ref).max() / scale:.2e}")
    return to_np(R)


def test_decorrelate_spd_host_and_odd_k():
    rng = np.random.default_rng(3)
    _check(_spd(72, 1, 1e6), rng.standard_normal((5, 72)), device=False)
    _check(_spd(73, 2, 1e4), rng.standard_normal((2, 73)), device=False)
    _check(np.array([[4.0]]), np.array([[2.0]]), device=False)


def test_decorrelate_device_k200():
    rng = np.random.default_rng(4)
    _check(_spd(200, 5, 1e6), rng.standard_normal((3, 200)), device=True, tol=1e-10)


def test_decorrelate_rank_deficient_and_lower_triangle_only():
    rng = np.random.default_rng(6)
    B = rng.standard_normal((40, 30))
    F = B @ B.T                                   # rank 30: ten eigenvalues fall under the cutoff
    R = _check(F, None, device=False, tol=1e-9)
    P = R @ F @ R
    assert abs(np.trace(P) - 30.0) < 1e-8
    G = _spd(24, 7, 1e3)
    Gbad = np.tril(G) + np.triu(rng.standard_normal((24, 24)), 1)
    cf = _cf()
    _, Rg = cf.decorrelate(Gbad)
    np.testing.assert_allclose(Rg, qml.inverse_sqrt(G), rtol=0, atol=1e-10 * np.abs(Rg).max())


def test_decorrelate_qml_estimates():
    """The decorrelated estimates of a QML run: F^-1/2 (y - b) with the run's own F."""
    cf = _cf()
    p = tiny_healpix("TQU", nside=2, lmax=6, cut=0.3, lowrank=2)
    bins = I.uniform_bins(2, 6, 2, ("TT", "EE", "BB", "TE"))
    maps = np.random.default_rng(11).standard_normal((2, p.n))
    out = cf.qml(p, bins, maps)
    F, q = out["F"], out["y"] - out["bias"][None, :]
    dec, _ = cf.decorrelate(F, q)
    ref = qml.decorrelate(F, q)
    np.testing.assert_allclose(dec, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
