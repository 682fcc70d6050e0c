"""GPU parity of the joint two-map QML (cf_qml_joint, Eq. C_joint) against the oracle's dense joint
estimator: F, y, noise bias and C_hat at 1e-10 (relative / in Fisher units, the FP64 bar), with
noise shared between the data sets (asymmetric N12) and without it, for T, QU and TQU."""
import copy

import numpy as np
import pytest

from oracle import qml
from paper_2605_21149_amd import cf
from paper_2605_21149_amd import inputs as I

from gpu_common import metric_chat, metric_F, metric_vec_fisher, say, to_np
from oracle_cases import tiny_healpix

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    cf.lib()
    assert torch.cuda.is_available(), "GPU tests selected but torch sees no GPU"


def _pair(fields, nside, lmax, shared, seed=31):
    p1 = tiny_healpix(fields, nside=nside, lmax=lmax, cut=0.25, lowrank=2)
    p2 = copy.copy(p1)
    rng = np.random.default_rng(seed)
    p2.noise_diag = p1.noise_diag * rng.uniform(0.5, 2.0, p1.n)
    N12 = None
    if shared:
        A = p1.noise_U
        B = A @ (0.8 * np.eye(A.shape[1]) + 0.3 * rng.standard_normal((A.shape[1], A.shape[1])))
        p2.noise_U = B
        N12 = A @ B.T                                   # not symmetric
    else:
        p2.noise_U = None
    return p1, p2, N12


def _case(fields, nside, lmax, lo, hi, shared, nmaps=2, device=True):
    p1, p2, N12 = _pair(fields, nside, lmax, shared)
    spectra = I.spectra_for_fields(fields)
    rng = np.random.default_rng(5)
    d1, d2 = rng.standard_normal((nmaps, p1.n)), rng.standard_normal((nmaps, p1.n))
    ref = qml.joint_dense(p1, p2, spectra, lo, hi, d1, d2, N12=N12)
    bins = I.Bins(np.asarray(lo, np.int32), np.asarray(hi, np.int32), tuple(spectra))
    got = {k: to_np(v) for k, v in cf.qml_joint(p1, p2, bins, d1, d2, N12=N12, device=device).items()}
    F = ref["F"]
    res = {"F": metric_F(got["F"], F), "y": metric_vec_fisher(got["y"], ref["y"], F),
           "bias": metric_vec_fisher(got["bias"], ref["bias"], F),
           "chat": metric_chat(got["chat"], ref["chat"], F)}
    return res, got


@pytest.mark.parametrize("fields", ["T", "QU", "TQU"])
def test_joint_shared_noise_matches_oracle(fields):
    say("joint qml:", fields, "nside 4, shared noise N12 = A B^T, device arrays")
    res, got = _case(fields, 4, 9, [2, 4, 6], [3, 5, 9], shared=True)
    say("  metrics", res)
    assert max(res.values()) < TOL
    np.testing.assert_allclose(got["F"], got["F"].T, rtol=0, atol=1e-14 * np.abs(got["F"]).max())


def test_joint_independent_noise_host_arrays():
    say("joint qml: QU nside 4, N12 = NULL, host arrays, 3 maps")
    res, _ = _case("QU", 4, 9, [2, 5], [4, 9], shared=False, nmaps=3, device=False)
    say("  metrics", res)
    assert max(res.values()) < TOL


def test_joint_qu_nside8_ragged():
    """A larger joint system (2n = 2 x 2 x 640ish: several 64-blocks and a ragged tail)."""
    say("joint qml: QU nside 8, shared noise")
    res, _ = _case("QU", 8, 17, [2, 6, 10, 14], [5, 9, 13, 17], shared=True)
    say("  metrics", res)
    assert max(res.values()) < TOL


def test_joint_rejects_mismatched_data_sets():
    p1, p2, _ = _pair("QU", 2, 6, shared=False)
    p3 = tiny_healpix("T", nside=2, lmax=6, cut=0.25)
    bins = I.Bins(np.array([2], np.int32), np.array([4], np.int32), ("EE",))
    d = np.zeros((1, p1.n))
    with pytest.raises(cf.CFError):
        cf.qml_joint(p1, p3, bins, d, np.zeros((1, p3.n)), device=False)
