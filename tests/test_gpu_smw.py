"""GPU parity of the harmonic-basis likelihood with multipole switching (cf_smw_*): against the
oracle's SMW likelihood on small problems (every window mode, a ragged last batch), and at the
full sizes of the scan workloads against the direct likelihood (the pixel-space scan of
cf_loglike_batch, itself checked against the oracle, and the oracle's direct likelihood at a
sampled point)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import likelihood, smw  # noqa: E402
from paper_2605_21149_amd import inputs as I  # noqa: E402
from gpu_common import say, to_np  # noqa: E402
from oracle_cases import random_spectra, tiny_healpix  # noqa: E402

pytestmark = pytest.mark.gpu
# Full-size tolerance (relative, -2 ln L and ln|C|): the FP64 solves against N_eff carry relative
# errors up to about n u kappa(N_eff) (n <= 5952, kappa about 1.2e4: 8e-9), and the data term's
# subtraction d^T N_eff^-1 d - |L^-1 b'|^2 amplifies them by about 1.3 on these workloads.
RTOL = 1e-8


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    from paper_2605_21149_amd import cf
    cf.lib()
    assert torch.cuda.is_available(), "GPU tests selected but torch sees no GPU"


def _cf():
    from paper_2605_21149_amd import cf
    return cf


def _points(p, seeds):
    """Point spectra: random positive-definite spectra (the window's entries are what matter)."""
    return np.stack([random_spectra(p.lmax, s) for s in seeds])


def _against_oracle(p, maps, pts, wlo, whi, wf, device):
    cf = _cf()
    with cf.SMW(p, maps, (wlo, whi), wf, device=device) as h:
        out = h.loglike(pts)
    got = {k: to_np(v) for k, v in out.items()}
    for i, cl in enumerate(pts):
        m2, chi2, ld = smw.smw_minus2lnL(p, maps, cl, wlo, whi, wf)
        np.testing.assert_allclose(got["m2lnL"][i], m2, rtol=1e-9)
        np.testing.assert_allclose(got["chi2"][i], chi2, rtol=1e-9)
        np.testing.assert_allclose(got["logdet"][i], ld, rtol=1e-9, atol=1e-9)
    return got


def test_smw_tqu_all_fields_matches_oracle_ragged_batch():
    say("smw: tiny TQU, window [2, 4] TEB, 20 points (batches of 16 and 4), device arrays")
    p = tiny_healpix("TQU", nside=2, lmax=6, cut=0.3, lowrank=2)
    maps = np.random.default_rng(71).standard_normal((3, p.n))
    _against_oracle(p, maps, _points(p, range(100, 120)), 2, 4, "TEB", device=True)


def test_smw_qu_e_window_matches_oracle_host_arrays():
    say("smw: tiny QU, window [2, 5] E (EB = 0), 3 points, host arrays")
    p = tiny_healpix("QU", nside=2, lmax=6, cut=0.25)
    p.cl = p.cl.copy()
    p.cl[5] = 0.0
    maps = np.random.default_rng(73).standard_normal((2, p.n))
    pts = _points(p, (201, 202, 203))
    _against_oracle(p, maps, pts, 2, 5, "E", device=False)


def _no_tp_spectra(lmax, seed):
    cl = random_spectra(lmax, seed)
    cl[3] = 0.0                                     # TE
    cl[4] = 0.0                                     # TB
    return cl


def test_smw_field_blocks_match_oracle_and_fall_back_when_coupled():
    """App. field_blocks: a TQU problem with no TE, TB and diagonal noise has no T x (E,B) block in
    M, so the handle records two field groups and factorises K' as a T block and an E,B block; the
    results equal the oracle's dense SMW likelihood and its direct Cholesky likelihood at 1e-9.  A
    call with TE inside the window at one point factorises the dense K' (still exact); a problem
    whose low-rank noise spans T and Q, U keeps one group."""
    cf = _cf()
    p = tiny_healpix("TQU", nside=2, lmax=6, cut=0.3)
    p.cl = _no_tp_spectra(6, 91)
    maps = np.random.default_rng(92).standard_normal((3, p.n))
    pts = np.stack([_no_tp_spectra(6, s) for s in range(93, 100)])
    say("smw field blocks: tiny TQU, window [2, 4] TEB, TE = TB = 0, diagonal noise")
    with cf.SMW(p, maps, (2, 4), "TEB") as h:
        assert h.setup_report["ir_iters"] == 2
        got, rep = h.loglike(pts, report=True)
        assert rep["ir_iters"] == 2
        coupled = pts.copy()
        coupled[2, 3, 3] = 0.2 * np.sqrt(coupled[2, 0, 3] * coupled[2, 1, 3])
        got2, rep2 = h.loglike(coupled, report=True)
        assert rep2["ir_iters"] == 1
    for res, pp in ((got, pts), (got2, coupled)):
        for i, cl in enumerate(pp):
            m2, chi2, ld = smw.smw_minus2lnL(p, maps, cl, 2, 4, "TEB")
            np.testing.assert_allclose(to_np(res["m2lnL"])[i], m2, rtol=1e-9)
            np.testing.assert_allclose(to_np(res["logdet"])[i], ld, rtol=1e-9, atol=1e-9)
            d2, _, _ = likelihood.minus2lnL(p, maps, cl=smw.window_spectra(p, cl, 2, 4, "TEB"))
            np.testing.assert_allclose(to_np(res["m2lnL"])[i], d2, rtol=1e-9)
    q = tiny_healpix("TQU", nside=2, lmax=6, cut=0.3, lowrank=2)
    q.cl = p.cl
    with cf.SMW(q, maps, (2, 4), "TEB") as h:
        assert h.setup_report["ir_iters"] == 1


def test_smw_full_window_equals_direct_gpu_likelihood():
    say("smw: tiny QU, full window [lmin, lmax] EB (N_eff = N) vs cf_loglike_batch")
    cf = _cf()
    p = tiny_healpix("QU", nside=2, lmax=5, cut=0.25, lowrank=2)
    maps = np.random.default_rng(72).standard_normal((2, p.n))
    pts = _points(p, (301, 302))
    with cf.SMW(p, maps, (p.lmin, p.lmax), "EB") as h:
        got = to_np(h.loglike(pts)["m2lnL"])
    ref = to_np(cf.loglike_batch([p], pts[:, None], [maps])["m2lnL"])[:, 0, :]
    np.testing.assert_allclose(got, ref, rtol=1e-9)


def test_smw_rejects_coupled_window_and_indefinite_points():
    cf = _cf()
    p = tiny_healpix("TQU", nside=2, lmax=5, cut=0.3)
    maps = np.random.default_rng(74).standard_normal((1, p.n))
    with pytest.raises(cf.CFError) as e:
        cf.SMW(p, maps, (2, 3), "E")                       # TE couples T and E in the window
    assert e.value.status == cf.CF_EINVAL
    with cf.SMW(p, maps, (2, 3), "TEB") as h:
        bad = _points(p, (401,))
        bad[0, 3, 3] = 5.0 * np.sqrt(bad[0, 0, 3] * bad[0, 1, 3])   # |TE| > sqrt(TT EE) at l = 3
        with pytest.raises(cf.CFError) as e2:
            h.loglike(bad)
        assert e2.value.status == cf.CF_EINVAL


@pytest.mark.timeout(900)
def test_smw_qu_nside16_scan_full_size():
    """The QU N_side 16 scan problem (n = 3968) with the EE window l = 2..29 (896 modes), 64 maps:
    against the direct GPU scan on 8 points and the oracle's direct likelihood at one point, at 1e-8
    relative."""
    cf = _cf()
    import torch
    say("smw: QU N_side 16, window [2, 29] E, 64 maps, 8 points")
    p = I.qu_scan_problem(16)
    maps = I.white_maps(p.n, 64, 403, rms=3.0)
    pts = I.scan_spectra(I.scan_points(8, seed=401), p.cl)
    d_maps = torch.as_tensor(maps).cuda()
    d_pts = torch.as_tensor(np.ascontiguousarray(pts)).cuda()
    with cf.SMW(p, d_maps, (2, 29), "E", device=True) as h:
        assert h.dim == 896
        got = {k: to_np(v) for k, v in h.loglike(d_pts).items()}
    ref = cf.loglike_batch([p], d_pts[:, None].contiguous(), [d_maps], device=True)
    ref = {k: to_np(v) for k, v in ref.items()}
    d = np.abs(got["m2lnL"] - ref["m2lnL"][:, 0, :]).max() / np.abs(ref["m2lnL"]).min()
    say(f"  max rel |d(-2lnL)| vs direct GPU scan: {d:.3e}")
    assert d <= RTOL
    assert np.abs(got["logdet"] - ref["logdet"][:, 0]).max() <= RTOL * np.abs(ref["logdet"]).min()
    m2o, _, ldo = likelihood.minus2lnL(p, maps[:4], cl=pts[3])
    say(f"  max rel |d(-2lnL)| vs oracle direct at point 3: {np.abs(got['m2lnL'][3, :4] / m2o - 1).max():.3e}")
    np.testing.assert_allclose(got["m2lnL"][3, :4], m2o, rtol=RTOL, atol=0)
    np.testing.assert_allclose(got["logdet"][3], ldo, rtol=RTOL, atol=0)


@pytest.mark.timeout(900)
def test_smw_tqu_nside16_all_fields_full_size():
    """The TQU N_side 16 problem of the bench (n = 5952), window l = 2..29 on T, E, B (2688 modes,
    TE coupling T and E), 64 maps: against the direct GPU scan on 4 points at 1e-8 relative (the
    oracle's SMW likelihood of this window is compared in the headline tests)."""
    cf = _cf()
    import torch
    say("smw: TQU N_side 16, window [2, 29] TEB, 64 maps, 4 points")
    p = I.tqu_problem_nside16(dense_noise=True)
    maps = I.white_maps(p.n, 64, 403, rms=3.0)
    pts = I.scan_spectra(I.scan_points(4, seed=401), p.cl)
    d_maps = torch.as_tensor(maps).cuda()
    d_pts = torch.as_tensor(np.ascontiguousarray(pts)).cuda()
    pk = cf.pack_problem(p, device=True)
    with cf.SMW(p, d_maps, (2, 29), "TEB", device=True, packed=pk) as h:
        assert h.dim == 2688
        got = {k: to_np(v) for k, v in h.loglike(d_pts).items()}
    ref = cf.loglike_batch([p], d_pts[:, None].contiguous(), [d_maps], device=True, packed=[pk])
    ref = {k: to_np(v) for k, v in ref.items()}
    d = np.abs(got["m2lnL"] - ref["m2lnL"][:, 0, :]).max() / np.abs(ref["m2lnL"]).min()
    say(f"  max rel |d(-2lnL)| vs direct GPU scan: {d:.3e}")
    assert d <= RTOL
    assert np.abs(got["logdet"] - ref["logdet"][:, 0]).max() <= RTOL * np.abs(ref["logdet"]).min()


def test_loglike_auto_follows_the_selector_and_matches_the_direct_likelihood():
    """cf_loglike_auto: a scan of 12 points whose EE varies in l 2..4 of a QU problem takes the
    harmonic basis (a 21-mode kernel per point against a Cholesky of the pixel covariance); one point
    over the whole band takes the pixel basis.  Both equal cf_loglike_batch at 1e-9 relative."""
    cf = _cf()
    p = tiny_healpix("QU", nside=4, lmax=9, cut=0.25)
    p.cl = p.cl.copy()
    p.cl[5] = 0.0                                           # EB would couple E to the fixed B
    maps = np.random.default_rng(95).standard_normal((2, p.n))
    pts = np.repeat(p.cl[None], 12, axis=0)
    pts[:, 1, 2:5] *= np.random.default_rng(96).uniform(0.5, 1.5, (12, 3))
    say("loglike auto: harmonic choice", p.n)
    got = cf.loglike_auto(p, (2, 4), "E", pts, maps)
    assert got["choice"]["basis"] == "harmonic" and got["choice"]["k_win"] == 21
    ref = to_np(cf.loglike_batch([p], pts[:, None], [maps])["m2lnL"])[:, 0, :]
    np.testing.assert_allclose(to_np(got["m2lnL"]), ref, rtol=1e-9)
    say("loglike auto: pixel choice")
    one = _points(p, (97,))
    got1 = cf.loglike_auto(p, (p.lmin, p.lmax), "EB", one, maps)
    assert got1["choice"]["basis"] == "pixel"
    ref1 = to_np(cf.loglike_batch([p], one[:, None], [maps])["m2lnL"])[:, 0, :]
    np.testing.assert_allclose(to_np(got1["m2lnL"]), ref1, rtol=1e-9)


# ------------------------------------------------------------------ Fisher / QML in the SMW basis
def _smw_qml_case(p, spectra, lo, hi, window, nmaps=2, seed=5):
    """cf_smw_qml against the oracle's harmonic QML (all multipoles of [lmin, lmax] estimated
    through Z, the same bins) and against the pixel-space cf_qml on the same maps."""
    from oracle import covariance as cv
    from oracle import qml
    from gpu_common import metric_chat, metric_F, metric_vec_fisher
    cf = _cf()
    C = cv.total_covariance(p)
    Lc = np.linalg.cholesky(C)
    maps = (Lc @ np.random.default_rng(seed).standard_normal((p.n, nmaps))).T.copy()
    ref = qml.qml_harmonic(p, spectra, lo, hi, maps, C)
    bins = I.Bins(np.asarray(lo, np.int32), np.asarray(hi, np.int32), tuple(spectra))
    got = {k: to_np(v) for k, v in cf.smw_qml(p, window, bins, maps, device=True).items()}
    pix = {k: to_np(v) for k, v in cf.qml(p, bins, maps, device=True).items()}
    F = ref["F"]
    res = {"F": metric_F(got["F"], F), "y": metric_vec_fisher(got["y"], ref["y"], F),
           "bias": metric_vec_fisher(got["bias"], ref["bias"], F),
           "chat": metric_chat(got["chat"], ref["chat"], F)}
    vs_pix = {"F": metric_F(got["F"], pix["F"]), "y": metric_vec_fisher(got["y"], pix["y"], F),
              "bias": metric_vec_fisher(got["bias"], pix["bias"], F),
              "chat": metric_chat(got["chat"], pix["chat"], F)}
    return res, vs_pix, got


def test_smw_qml_masked_qu_windowed_noise():
    """Masked QU with low-rank noise; the window [2, 5] leaves l in [6, 9] at the fiducial inside
    N_eff: F, y, bias and C_hat at 1e-10 of the oracle and of the pixel-space estimator."""
    p = tiny_healpix("QU", nside=4, lmax=9, cut=0.25, lowrank=2)
    spectra = ("EE", "BB", "EB")
    say("smw qml: QU nside 4, window [2, 5], bins [2,3] [4,5]", p.n)
    res, vs_pix, got = _smw_qml_case(p, spectra, [2, 4], [3, 5], (2, 5))
    say("  vs oracle", res, "vs pixel", vs_pix)
    assert max(res.values()) < 1e-10
    assert max(vs_pix.values()) < 1e-10
    np.testing.assert_allclose(got["F"], got["F"].T, rtol=0, atol=1e-14 * np.max(np.abs(got["F"])))


@pytest.mark.parametrize("fields,window", [("T", (2, 7)), ("TQU", (2, 6))])
def test_smw_qml_other_fields(fields, window):
    p = tiny_healpix(fields, nside=4, lmax=9, cut=0.25, lowrank=2)
    spectra = I.spectra_for_fields(fields)
    lo = [2, 4, 5]; hi = [3, 4, window[1]]
    say("smw qml:", fields, "window", window, p.n)
    res, vs_pix, _ = _smw_qml_case(p, spectra, lo, hi, window, nmaps=3, seed=9)
    say("  vs oracle", res, "vs pixel", vs_pix)
    assert max(res.values()) < 1e-10
    assert max(vs_pix.values()) < 1e-10


def test_smw_qml_rejects_bins_outside_window():
    cf = _cf()
    p = tiny_healpix("T", nside=2, lmax=6, cut=0.3)
    bins = I.Bins(np.array([2, 5], np.int32), np.array([4, 6], np.int32), ("TT",))
    maps = np.zeros((1, p.n))
    with pytest.raises(cf.CFError):
        cf.smw_qml(p, (2, 4), bins, maps, device=True)
