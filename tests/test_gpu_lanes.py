"""Two calls at once on one device, from two host threads: the library gives each call a lane of
its own (streams, events, workspace, pinned flags), and once calls have overlapped it stops using
the CU-masked streams for single factorisations.  Neither may change a result: every output of
the overlapped calls must equal, bit for bit, the same calls made one after the other (before and
after the switch), and those agree with the oracle within the FP64 bar."""
import threading

import numpy as np
import pytest

from oracle import covariance as cv
from oracle import likelihood, qml
from paper_2605_21149_amd import cf
from paper_2605_21149_amd import inputs as I

from gpu_common import metric_F, metric_vec_fisher, say, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    cf.lib()
    assert torch.cuda.is_available(), "GPU tests selected but torch sees no GPU"


def test_fisher_qml_beside_a_likelihood_batch():
    import torch
    # Fisher + QML of the spin-0 N_side 8 problem (n = 544, unbinned TT, l 2..24) on one thread,
    # -2 ln L of the QU N_side 8 scan problem (n = 1088, 8 points x 16 maps) on the other
    pq = I.spin0_problem_nside8()
    lo = np.arange(2, 25).astype(np.int32)
    bins = I.Bins(lo, lo, ("TT",))
    C = cv.total_covariance(pq)
    maps_q = (np.linalg.cholesky(C) @ np.random.default_rng(101).standard_normal((pq.n, 1))).T
    pl = I.qu_scan_problem(8)
    maps_l = I.white_maps(pl.n, 16, 402, rms=3.0)
    clp = np.ascontiguousarray(I.scan_spectra(I.scan_points(8, seed=401), pl.cl)[:, None])
    pkq, pkl = cf.pack_problem(pq, device=True), cf.pack_problem(pl, device=True)
    dq = torch.as_tensor(np.ascontiguousarray(maps_q)).cuda()
    dl = torch.as_tensor(maps_l).cuda()
    dcl = torch.as_tensor(clp).cuda()
    sA, sB = torch.cuda.Stream(), torch.cuda.Stream()

    def run_q():
        with torch.cuda.stream(sA):
            r = cf.qml(pq, bins, dq, device=True, packed=pkq)
            sA.synchronize()
        return {k: to_np(v) for k, v in r.items()}

    def run_l():
        with torch.cuda.stream(sB):
            r = cf.loglike_batch([pl], dcl, [dl], device=True, packed=[pkl])
            sB.synchronize()
        return {k: to_np(v) for k, v in r.items()}

    def at_once():
        box, err = {}, []

        def side():
            try:
                box["l"] = run_l()
            except BaseException as e:   # re-raised below
                err.append(e)
        th = threading.Thread(target=side)
        th.start()
        try:
            box["q"] = run_q()
        finally:
            th.join()
        if err:
            raise err[0]
        return box["q"], box["l"]

    say("lanes: sequential reference calls ...")
    q0, l0 = run_q(), run_l()
    ref = qml.qml_harmonic(pq, ("TT",), lo, lo, maps_q, C)
    assert metric_F(q0["F"], ref["F"]) < TOL
    assert metric_vec_fisher(q0["y"], ref["y"], ref["F"]) < TOL
    assert metric_vec_fisher(q0["bias"], ref["bias"], ref["F"]) < TOL
    for i in (0, 7):
        m2, _, ld = likelihood.minus2lnL(pl, maps_l, cl=clp[i, 0])
        assert np.max(np.abs(l0["m2lnL"][i, 0] - m2) / np.abs(m2)) < TOL
        assert abs(l0["logdet"][i, 0] - ld) <= TOL * abs(ld)
    for rep in range(3):
        say(f"lanes: overlapped calls, repetition {rep}")
        q, l = at_once()
        for k in q0:
            assert np.array_equal(q[k], q0[k]), k
        for k in l0:
            assert np.array_equal(l[k], l0[k]), k
    say("lanes: sequential calls after the overlap")
    q, l = run_q(), run_l()
    for k in q0:
        assert np.array_equal(q[k], q0[k]), k
    for k in l0:
        assert np.array_equal(l[k], l0[k]), k
