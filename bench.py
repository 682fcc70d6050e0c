"""Benchmark of the hot path on the TQU N_side = 16 workload (|b| > 20 deg mask, n = 5952,
l in [2, 47], 6 spectra x 12 bins of width 4, dense N = 2 I + U U^T with 20 smooth modes).

One step = one pass of the whole path on one batch of synthetic input:
  Fisher + QML of one map (covariance assembly, Cholesky, harmonic basis, triangular solves,
  Z = Y^T C^-1 Y, Fisher block reduction, y, noise bias, C_hat)
  + the likelihood -2 ln L of SCAN_POINTS parameter points x 64 maps (per point: covariance
    rebuild, Cholesky, log det, 64 triangular solves, chi^2).
The two parts run one after the other; with --overlap each timed step runs them at once, the
likelihood on a second host thread (the library gives concurrent calls separate streams and
workspaces), and the step ends when both have (measured slower on this workload: 29.0 against
27.7 ms per step).
Inputs are resident in device memory before the timed region.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

SCAN_POINTS = 8
NMAPS_SCAN = 64
PEAK_FP64_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 30 timed steps (under a second): the one instrumented step among them (per-launch GEMM
    # events, about 2 ms of extra host time with the device idle) then adds under 0.1 ms per step
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--overlap", action="store_true",
                    help="run the step's two parts at once on two host threads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="time the oracle sample as a median of 3 after one warmup, plus a single-thread run")
    ap.add_argument("--scan-points", type=int, default=8192,
                    help="points of the two-problem QU scan (N_side 8 + 16, 64 maps each)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32 / BF16x3 comparison")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (HBM counter calibration)")
    ap.add_argument("--tune-cache", default="", metavar="PATH",
                    help="autotuning table to use (default: a fresh one, tuned during warmup)")
    ap.add_argument("--no-smw", action="store_true",
                    help="skip the harmonic-basis (SMW, multipole switching) likelihood measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the cross-QML and decorrelated-normalisation timings")
    ap.add_argument("--smw-only", action="store_true",
                    help="only run the SMW likelihood measurement and print its JSON")
    ap.add_argument("--no-emulator", action="store_true",
                    help="skip training and measuring the likelihood emulator on the QU N_side 16 scan problem")
    ap.add_argument("--emu-train", type=int, default=65536, help="exact training points")
    ap.add_argument("--emu-epochs", type=int, default=100)
    ap.add_argument("--emu-query", type=int, default=65536)
    return ap.parse_args()


GEMM_ROLE = {"0": "(triangular solves and panel updates)", "1": "(Z = G^T G, E,B block)",
             "2": "(Cholesky updates C -= L L^T)"}


def _traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when that
    summary was taken on a different source of the GEMM kernel than the one built here."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "traffic_tqu_nside16.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(here, "paper_2605_21149_amd", "csrc", "gemm.hip"), "rb").read()
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel.replace(" ", ""))
    if not k or rec.get("gemm_source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def _tuned_lines(path):
    """The autotuner's entries (launch shapes chosen during warmup and tuning calls)."""
    try:
        return [l.strip() for l in open(path) if l.startswith("scan ")]
    except OSError:
        return None


def _tuned_line(path, n=None):
    lines = [l for l in (_tuned_lines(path) or []) if n is None or f" n={n} " in l]
    return lines[-1] if lines else None


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def emulator_bench(cf, I, n_train, epochs, n_query, spread_max=0.1, seed_map=403):
    """Emulator of -2 ln L on the QU N_side 16 scan problem (n = 3968, 7 parameters: EE band
    amplitudes over l 2..29 and the reionisation bump, all inside the E window l 2..29), map 0.
    The fastest exact likelihood there is the harmonic-basis handle of that window (cf_smw_*), which
    also generates the training data and answers the fallbacks; the pixel-space scan is timed on a
    short sample for comparison.  Queries: 90 % in the parameter box, 10 % from [0.4, 1.6]^7.
    Accuracy: every emulated query against the exact value from the same handle."""
    import torch
    dev = torch.device("cuda:0")
    p = I.qu_scan_problem(16)
    n = p.n
    dmap = I.white_maps(n, 1, seed_map, rms=3.0)[0]
    base = I.scan_spectra(np.zeros((1, 7)), p.cl)[0]
    basis = np.stack([I.scan_spectra(np.eye(7)[k:k + 1], p.cl)[0] - base for k in range(7)])
    packed = cf.pack_problem(p, device=True)
    d_map = torch.as_tensor(dmap).to(dev)

    def spectra(x):
        return torch.as_tensor(np.ascontiguousarray(base[None] + np.einsum("nk,kxl->nxl", x, basis))).to(dev)

    # pixel-space scan, short sample (the batch shape tunes on a first, untimed call of the same
    # size: a call that could batch more points than the tuning trials would tune again)
    xd = I.scan_points(512, seed=500)
    cf.loglike_batch([p], spectra(xd)[:, None], [d_map[None]], device=True, packed=[packed], autotune=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cf.loglike_batch([p], spectra(xd)[:, None], [d_map[None]], device=True, packed=[packed], autotune=True)
    torch.cuda.synchronize()
    direct_rate = len(xd) / (time.perf_counter() - t0)
    with cf.SMW(p, d_map, (2, 29), "E", device=True) as h:
        def exact(x):
            out = []
            for i in range(0, len(x), 16384):
                out.append(h.loglike(spectra(x[i:i + 16384]))["m2lnL"][:, 0])
            return torch.cat(out)
        exact(I.scan_points(1024, seed=499))
        torch.cuda.synchronize()
        xt = I.scan_points(n_train, seed=501)
        t0 = time.perf_counter()
        yt = exact(xt)
        torch.cuda.synchronize()
        t_gen = time.perf_counter() - t0
        smw_rate = n_train / t_gen
        _log(f"emulator: {n_train} exact points (harmonic-basis handle) in {t_gen:.1f} s")
        emu = cf.Emulator(7, 256, 3, 4, seed=502)
        tr = emu.train(torch.as_tensor(xt).to(dev), yt, epochs=epochs, batch=1024, device=True, report=True)
        _log(f"emulator: trained {tr['ir_iters']} steps in {tr['ms_total'] / 1e3:.1f} s, held-out rms "
             f"{tr['est_err'][1]:.4f}")
        nin = int(round(0.9 * n_query))
        q = np.concatenate([I.scan_points(nin, seed=506), I.scan_points(n_query - nin, seed=507, lo=0.4, hi=1.6)])
        d_q = torch.as_tensor(q).to(dev)
        emu.predict(d_q[:4096], spread_max=spread_max, device=True, exact_smw=(h, base, basis))   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r_only, rep_only = emu.predict(d_q, spread_max=spread_max, device=True, report=True)
        torch.cuda.synchronize()
        t_only = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = emu.predict(d_q, spread_max=spread_max, device=True, exact_smw=(h, base, basis))
        torch.cuda.synchronize()
        t_fb = time.perf_counter() - t0
        t0 = time.perf_counter()
        ex = exact(q)
        torch.cuda.synchronize()
        t_ex = time.perf_counter() - t0
    fb = r["fallback"].cpu().numpy().astype(bool)
    err = np.abs(r["y"].cpu().numpy() - ex.cpu().numpy())
    emu_err = err[~fb] if (~fb).any() else np.zeros(1)
    _log(f"emulator: {fb.mean():.3f} fallback, predict {t_fb:.2f} s")
    return {
        "problem": f"QU N_side 16 scan (n={n}), 7 parameters inside the E window l 2..29, map 0",
        "target_std": float(yt.std().item()),
        "network": "7-256-256-256-1 SiLU, 4 members, BF16 MFMA hidden products / FP32 accumulate",
        "train_points": n_train, "epochs": epochs, "train_steps": tr["ir_iters"],
        "train_source": "harmonic-basis (SMW) handle of the window, FP64",
        "exact_gen_s": t_gen,
        "train_s": tr["ms_total"] / 1e3, "train_tflops": tr["flops"] / (tr["ms_total"] * 1e-3) / 1e12,
        "heldout_rms": tr["est_err"][1], "heldout_max": tr["est_err"][2], "heldout_spread": tr["est_err"][3],
        "queries": n_query, "spread_max": spread_max, "fallback_frac": float(fb.mean()),
        "exact_pixel_points_per_s": direct_rate,
        "exact_smw_points_per_s": len(q) / t_ex,
        "ensemble_only_evals_per_s": n_query / t_only,
        "ensemble_kernel_ms": rep_only["est_err"][0],
        "evals_per_s_with_fallback": n_query / t_fb,
        "gain_vs_fastest_exact": (n_query / t_fb) / (len(q) / t_ex),
        "gain_vs_pixel_exact": (n_query / t_fb) / direct_rate,
        "abs_err_emulated": {"p50": float(np.median(emu_err)), "p99": float(np.quantile(emu_err, 0.99)),
                              "max": float(emu_err.max()), "count": int((~fb).sum())},
        "abs_err_fallback_max": float(err[fb].max()) if fb.any() else 0.0,
    }


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample(problem, bins, cl_points, maps_qml, maps_scan):
    """One Fisher + QML pass of the oracle in full (covariance, factorisation, Z, all 72 x 72
    Fisher entries, y, bias, C_hat) and one likelihood point (covariance rebuild, Cholesky, 64
    maps); returns (seconds of the Fisher + QML pass, seconds of the likelihood point)."""
    import scipy.linalg as sla
    from oracle import covariance as cv, likelihood, qml
    import copy
    t0 = time.perf_counter()
    C = cv.total_covariance(problem)
    Z, Y, modes, fac = qml.projected_inverse(problem, C)
    coo = qml.coo_derivatives(problem, modes, bins.spectra, bins.lo, bins.hi)
    F = qml.fisher_from_z(Z, coo)
    w = (Y.T @ sla.cho_solve(fac, maps_qml.T)).T
    y = qml.quadratic_from_w(w, coo)
    np.linalg.solve(F, np.atleast_2d(y).T)
    t_fisher = time.perf_counter() - t0
    t0 = time.perf_counter()
    p1 = copy.copy(problem)
    p1.cl = cl_points[0, 0]
    likelihood.chi2_logdet(cv.total_covariance(p1), maps_scan)
    t_point = time.perf_counter() - t0
    return t_fisher, t_point


def cpu_baseline(problem, bins, cl_points, maps_qml, maps_scan, full=False):
    """The CPU oracle on the host cores: the Fisher + QML pass timed in full and one of the
    SCAN_POINTS likelihood points timed and scaled to the step.  full: one warmup, the median of
    three runs, and one run on a single BLAS thread."""
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    if full:
        _oracle_sample(problem, bins, cl_points, maps_qml, maps_scan)
        _log("cpu baseline: warmup run done")
        runs = []
        for r in range(3):
            runs.append(_oracle_sample(problem, bins, cl_points, maps_qml, maps_scan))
            _log(f"cpu baseline: run {r + 1} of 3: Fisher+QML {runs[-1][0]:.1f} s, one point {runs[-1][1]:.1f} s")
        t_f = float(np.median([r[0] for r in runs]))
        t_p = float(np.median([r[1] for r in runs]))
    else:
        t_f, t_p = _oracle_sample(problem, bins, cl_points, maps_qml, maps_scan)
    step = t_f + SCAN_POINTS * t_p
    out = {"value": 1.0 / step, "unit": "steps/s", "cores": int(threads), "kind": "oracle",
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
           "fisher_qml_s": t_f, "loglike_point_s": t_p,
           "sample": (f"one Fisher+QML pass timed in full ({t_f:.1f} s: covariance, Cholesky, Z, all 72x72 "
                      f"Fisher entries, y, bias, C_hat) and one of {SCAN_POINTS} likelihood points "
                      f"({t_p:.1f} s, 64 maps) scaled by {SCAN_POINTS}; "
                      + ("median of 3 after one warmup" if full else "one run")
                      + f"; host BLAS threads {threads}")}
    if full:
        with threadpool_limits(limits=1):
            t1f, t1p = _oracle_sample(problem, bins, cl_points, maps_qml, maps_scan)
        _log(f"cpu baseline: single thread: Fisher+QML {t1f:.1f} s, one point {t1p:.1f} s")
        out["single_thread"] = {"fisher_qml_s": t1f, "loglike_point_s": t1p,
                                "steps_per_s": 1.0 / (t1f + SCAN_POINTS * t1p)}
    return out


def smw_section(cf, I, problem, packed, d_maps_scan, direct_m2, direct_pts_per_s, reps=3):
    """Harmonic-basis likelihood with multipole switching (cf_smw_*): the EE window l = 2..29 of the
    scan model, on all fields of the TQU problem (TE couples T and E) and on E alone for the QU
    N_side 16 scan problem.  Setup = N_eff factorisation with the maps' and the window's solves;
    the scan rate counts every point's K' build, factorisation and log det.  Accuracy: the largest
    |d(-2 ln L)| against the direct pixel-space scan at the step's points.  Points per call: 64 for
    the TQU window (2688 modes; the library's batches hold about 100 points), 512 for the E window
    (896 modes; batches of 128), bounded samples of the scans' parameter box."""
    import torch
    out = {}
    cases = [("tqu_nside16", problem, packed, d_maps_scan, "TEB", 64),
             ("qu_nside16", I.qu_scan_problem(16), None, None, "E", 512)]
    for name, p, pk, d_maps, wf, npoints in cases:
        pk = pk or cf.pack_problem(p, device=True)
        if d_maps is None:
            d_maps = torch.as_tensor(I.white_maps(p.n, NMAPS_SCAN, 403, rms=3.0)).cuda()
        pts = torch.as_tensor(np.ascontiguousarray(I.scan_spectra(I.scan_points(npoints, seed=401), p.cl))).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = cf.SMW(p, d_maps, (2, 29), wf, device=True, packed=pk)
        torch.cuda.synchronize()
        setup_ms = 1e3 * (time.perf_counter() - t0)
        h.loglike(pts[:SCAN_POINTS])
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = h.loglike(pts)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        k = h.dim
        flops = k ** 3 / 3.0 + k * k * NMAPS_SCAN     # per point: factorisation of [K'; b'^T]
        rec = {"window": f"l 2-29, fields {wf}", "k_win": k, "n": p.n, "setup_ms": setup_ms,
               "points": npoints, "scan_ms": 1e3 * min(ts), "points_per_s": npoints / min(ts),
               "map_evals_per_s": npoints * NMAPS_SCAN / min(ts),
               "achieved_tflops": npoints * flops / min(ts) / 1e12}
        if name == "tqu_nside16":
            got = res["m2lnL"][:SCAN_POINTS].cpu().numpy()
            rec["max_abs_dm2lnL_vs_direct"] = float(np.abs(got - direct_m2).max())
            rec["direct_points_per_s"] = direct_pts_per_s
        h.close()
        out[name] = rec
    return out


def qml_extras(cf, I, problem, bins, packed, d_maps_qml, reps=3):
    """Cross-QML of the TQU problem with a second data set (same model, diagonal noise of 2 to
    4 uK^2, one map pair), the decorrelated normalisation of the step's QML estimates (K = 72):
    median device-synchronised wall times; and iterative QML of the step's map (one run)."""
    import copy
    import torch
    p2 = copy.copy(problem)
    p2.noise_dense = np.diag(np.random.default_rng(31).uniform(2.0, 4.0, problem.n))
    pk2 = cf.pack_problem(p2, device=True)
    d_maps2 = torch.as_tensor(I.white_maps(problem.n, 1, 203, rms=3.0)).cuda()
    tc, td, sweeps = [], [], 0
    out = None
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = cf.qml_cross(problem, p2, bins, d_maps_qml, d_maps2, device=True, packed=(packed, pk2))
        torch.cuda.synchronize()
        tc.append(time.perf_counter() - t0)
    q = cf.qml(problem, bins, d_maps_qml, device=True, packed=packed)
    qq = q["y"] - q["bias"][None, :]
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        (_, _), rep = cf.decorrelate(q["F"], qq, device=True, report=True)
        torch.cuda.synchronize()
        td.append(time.perf_counter() - t0)
        sweeps = rep["ir_iters"]
    W = out["W"].cpu().numpy()
    # iterative QML of the step's map from the fiducial, to 1e-6 Fisher errors
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = cf.qml_iterate(problem, bins, d_maps_qml[0], max_iter=40, tol=1e-6, device=True, packed=packed)
    torch.cuda.synchronize()
    ti = time.perf_counter() - t0
    return {"cross_qml": {"ms": 1e3 * float(np.median(tc[1:])), "n": problem.n, "K": int(W.shape[0]),
                          "W_min_eigenvalue_over_max": float(np.linalg.eigvalsh(W).min() / np.linalg.eigvalsh(W).max())},
            "decorrelate": {"ms": 1e3 * float(np.median(td[1:])), "K": int(qq.shape[1]), "jacobi_sweeps": int(sweeps)},
            "qml_iterate": {"ms": 1e3 * ti, "iterations": it["iterations"], "tol_fisher_errors": 1e-6}}


def qu_scan(cf, I, npoints=8192):
    """The QU likelihood scan of the batched-scan workload (N_side 8, n = 1088, and N_side 16,
    n = 3968, 64 maps each) over npoints points of its parameter box, each problem in its own call
    (calls that mix the two problems stay off the GPU: see the library's notes) in the launch shape
    the autotuner recorded for it (tuned on 128 points first): points/s (one point = both problems,
    the two calls' times added) and map evaluations/s, FP64 and FP32 mixed (with the refined chi^2
    and the log-det correction), and the mixed path's largest |d(-2 ln L)| against FP64."""
    import torch
    pa, pb = I.qu_scan_problem(8), I.qu_scan_problem(16)
    pks = [cf.pack_problem(pa, device=True), cf.pack_problem(pb, device=True)]
    maps = [torch.as_tensor(I.white_maps(pa.n, 64, 402, rms=3.0)).cuda(),
            torch.as_tensor(I.white_maps(pb.n, 64, 403, rms=3.0)).cuda()]
    pts = I.scan_points(npoints, seed=401)
    clp = np.zeros((npoints, 2, 6, pb.lmax + 1))
    clp[:, 0, :, :pa.lmax + 1] = I.scan_spectra(pts, pa.cl)
    clp[:, 1] = I.scan_spectra(pts, pb.cl)
    d_cl = torch.as_tensor(clp).cuda()
    out, ref = {"n": [pa.n, pb.n], "points": npoints, "maps": 64}, None
    for prec, name in ((cf.CF_FP64, "fp64"), (cf.CF_MIXED_FP32, "fp32")):
        for k, p in enumerate((pa, pb)):
            cf.loglike_batch([p], d_cl[:128, k:k + 1, :, :p.lmax + 1].contiguous(), maps[k:k + 1], precision=prec,
                             device=True, packed=pks[k:k + 1], autotune=True)
        t, parts, tk = 0.0, [], []
        for k, p in enumerate((pa, pb)):
            cl1 = d_cl[:, k:k + 1, :, :p.lmax + 1].contiguous()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = cf.loglike_batch([p], cl1, maps[k:k + 1], precision=prec, device=True, packed=pks[k:k + 1],
                                   autotune=True)
            torch.cuda.synchronize()
            tk.append(time.perf_counter() - t0)
            t += tk[-1]
            parts.append(res["m2lnL"].cpu().numpy())
        _log(f"qu scan {name}: {npoints} points x 2 problems in {t:.2f} s")
        m2 = np.concatenate(parts, axis=1)
        out[name] = {"ms": 1e3 * t, "ms_per_problem": [1e3 * x for x in tk], "points_per_s": npoints / t,
                     "map_evals_per_s": 2 * 64 * npoints / t}
        if ref is None:
            ref = m2
        else:
            out[name]["max_abs_dm2lnL_vs_fp64"] = float(np.abs(m2 - ref).max())
    out["autotuned"] = [l for l in (_tuned_lines(os.environ["CF_TUNE_CACHE"]) or [])
                        if f"n={pa.n} " in l or f"n={pb.n} " in l]
    return out


def tqu_scan(cf, I, problem, packed, d_maps_scan, npoints=64):
    """The likelihood of the step's workload as a scan: npoints points per call (the step itself
    holds 8 per call) in the launch shape the autotuner picks for them, 64 maps, FP64: points/s and
    map evaluations/s, median of three calls after the tuning call."""
    import torch
    pts = I.scan_points(npoints, seed=404)
    cl = torch.as_tensor(np.ascontiguousarray(I.scan_spectra(pts, problem.cl)[:, None])).cuda()
    cf.loglike_batch([problem], cl, [d_maps_scan], device=True, packed=[packed], autotune=True)
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cf.loglike_batch([problem], cl, [d_maps_scan], device=True, packed=[packed], autotune=True)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    n = problem.n
    return {"points_per_call": npoints, "ms": 1e3 * t, "points_per_s": npoints / t,
            "map_evals_per_s": npoints * NMAPS_SCAN / t,
            "tflops": npoints * (n ** 3 / 3.0 + NMAPS_SCAN * n ** 2) / t / 1e12,
            "autotuned": [l for l in (_tuned_lines(os.environ["CF_TUNE_CACHE"]) or []) if f"n={n} " in l]}


def other_fishers(cf, I, reps=2):
    """Fisher+QML of one map for the two other QML workloads, median device-synchronised wall time:
    the spin-0 N_side 8 problem (n = 544, 23 unbinned multipoles; latency-bound) in FP64, and the
    QU N_side 32 problem (n = 12288, 18424 modes, EE, BB, EB unbinned over l = 2..95, K = 282) in
    FP64 and in the FP32 mixed path, with the mixed path's F error against FP64."""
    import torch
    out = {}
    for name, p, spectra, precs in (
            ("t_nside8", I.spin0_problem_nside8(), ("TT",), (cf.CF_FP64,)),
            ("qu_nside32", I.qu_problem_nside32(), ("EE", "BB", "EB"), (cf.CF_FP64, cf.CF_MIXED_FP32))):
        bins = I.uniform_bins(p.lmin, p.lmax, 1, spectra)
        pk = cf.pack_problem(p, device=True)
        d = torch.as_tensor(I.white_maps(p.n, 1, 302, rms=1.0)).cuda()
        rec, ref = {"n": p.n, "K": len(spectra) * (p.lmax - p.lmin + 1)}, None
        for prec in precs:
            ts, res = [], None
            for _ in range(reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = cf.qml(p, bins, d, precision=prec, device=True, packed=pk)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            key = "fp64_ms" if prec == cf.CF_FP64 else "fp32_ms"
            rec[key] = 1e3 * float(np.median(ts[1:]))
            F = res["F"].cpu().numpy()
            if ref is None:
                ref = F
            else:
                rec["fp32_err_F_relfro"] = float(np.linalg.norm(F - ref) / np.linalg.norm(ref))
        out[name] = rec
        del pk, d
        torch.cuda.empty_cache()
    return out


def mixed_precision(cf, I, problem, bins, packed, d_maps_qml, d_cl, d_maps_scan, reps=3):
    """Fisher+QML and likelihood-batch times for FP64, FP32-MFMA and split-BF16x3 paths, with the
    errors of the mixed results against the FP64 path (F: relative Frobenius; y, b: in units of
    the Fisher errors; -2lnL: absolute)."""
    import torch
    out = {}
    base = None
    for prec, name in ((cf.CF_FP64, "fp64"), (cf.CF_MIXED_FP32, "fp32"), (cf.CF_MIXED_BF16X3, "bf16x3")):
        tq, tl = [], []
        for _ in range(reps):
            torch.cuda.synchronize(); t = time.perf_counter()
            q = cf.qml(problem, bins, d_maps_qml, precision=prec, device=True, packed=packed)
            torch.cuda.synchronize(); tq.append(time.perf_counter() - t)
            t = time.perf_counter()
            l = cf.loglike_batch([problem], d_cl, [d_maps_scan], precision=prec, device=True, packed=[packed])
            torch.cuda.synchronize(); tl.append(time.perf_counter() - t)
        q = {k: v.cpu().numpy() for k, v in q.items()}
        l = {k: v.cpu().numpy() for k, v in l.items()}
        rec = {"fisher_qml_ms": 1e3 * float(np.median(tq)), "loglike_ms": 1e3 * float(np.median(tl))}
        if base is None:
            base = (q, l)
        else:
            F = base[0]["F"]
            d = np.sqrt(np.diag(F))
            rec["err_F_relfro"] = float(np.linalg.norm(q["F"] - F) / np.linalg.norm(F))
            rec["err_y"] = float(np.max(np.abs(q["y"] - base[0]["y"]) / d))
            rec["err_bias"] = float(np.max(np.abs(q["bias"] - base[0]["bias"]) / d))
            rec["err_m2lnL_abs"] = float(np.max(np.abs(l["m2lnL"] - base[1]["m2lnL"])))
            rec["err_chi2_abs"] = float(np.max(np.abs(l["chi2"] - base[1]["chi2"])))
        out[name] = rec
    return out


def host_input_step(cf, problem, bins, maps_qml, maps_scan, cl_points, steps=3):
    """The same step with every input in host memory (numpy arrays, mem = CF_MEM_HOST): the library
    copies the dense noise covariance, the maps and the scan spectra to the device on each call and
    the results back, so this rate includes the PCIe transfers.  Reported beside the device-resident
    rate, never as the bench value."""
    import torch
    pk = cf.pack_problem(problem, device=False)
    cl = np.ascontiguousarray(cl_points)

    def step():
        cf.qml(problem, bins, maps_qml, packed=pk)
        cf.loglike_batch([problem], cl, [maps_scan], packed=[pk], autotune=True)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    return {"steps": steps, "ms_per_step": ms, "steps_per_s": 1e3 / ms,
            "bytes_in_per_step": int(2 * problem.n * problem.n * 8 + maps_qml.size * 8 + maps_scan.size * 8
                                     + cl.size * 8)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the path runs on a single GPU; sharding the scan points or the Y columns across "
              f"GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.calibrate_copy:
        n = args.calibrate_copy << 17                     # doubles
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 8 * n}), flush=True)
        return
    # a fresh autotuning table: the first warmup step tunes the likelihood batch of this workload
    if args.tune_cache:
        os.environ["CF_TUNE_CACHE"] = args.tune_cache
    else:
        import tempfile
        os.environ["CF_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="cf_bench_"), "autotune.txt")
    from paper_2605_21149_amd import cf
    from paper_2605_21149_amd import inputs as I

    dev = torch.device("cuda:0")
    problem = I.tqu_problem_nside16(dense_noise=True)
    bins = I.uniform_bins(2, 47, 4, I.SPEC_NAMES)
    n = problem.n
    maps_qml = I.white_maps(n, 1, 202, rms=3.0)
    maps_scan = I.white_maps(n, NMAPS_SCAN, 403, rms=3.0)
    pts = I.scan_points(SCAN_POINTS, seed=401)
    cl_points = I.scan_spectra(pts, problem.cl)[:, None]      # [P][1][6][48]
    # device-resident inputs
    packed = cf.pack_problem(problem, device=True)
    d_maps_qml = torch.as_tensor(maps_qml).to(dev)
    d_maps_scan = torch.as_tensor(maps_scan).to(dev)
    d_cl = torch.as_tensor(np.ascontiguousarray(cl_points)).to(dev)
    torch.cuda.synchronize()
    if args.smw_only:
        direct = cf.loglike_batch([problem], d_cl, [d_maps_scan], device=True, packed=[packed])
        print(json.dumps({"smw": smw_section(cf, I, problem, packed, d_maps_scan,
                                             direct["m2lnL"][:, 0, :].cpu().numpy(), None)}), flush=True)
        return

    sA, sB = torch.cuda.Stream(), torch.cuda.Stream()   # default priority, one per part

    def parts(timed, overlap):
        """One step: Fisher + QML of one map on this thread, the likelihood batch on this thread
        after it (overlap False) or on a second thread at the same time (overlap True).  Returns
        the two reports and each part's wall time (host call until its stream is idle)."""
        out, err = {}, []

        def lik():
            try:
                with torch.cuda.stream(sB):
                    t = time.perf_counter()
                    # in the launch shape the autotuner chose before warmup (eager launches here)
                    rep = cf.loglike_batch([problem], d_cl, [d_maps_scan], device=True, report=True,
                                           stage_timing=timed, packed=[packed], autotune=True)[1]
                    sB.synchronize()
                    out["l"] = (rep, time.perf_counter() - t)
            except BaseException as e:      # re-raised on the calling thread
                err.append(e)
        th = threading.Thread(target=lik) if overlap else None
        if th:
            th.start()
        try:
            with torch.cuda.stream(sA):
                t = time.perf_counter()
                rep = cf.qml(problem, bins, d_maps_qml, device=True, stage_timing=timed, report=True,
                             packed=packed)[1]
                sA.synchronize()
                out["q"] = (rep, time.perf_counter() - t)
        finally:
            if th:
                th.join()
        if not th:
            lik()
        if err:
            raise err[0]
        return out["q"], out["l"]

    overlap = args.overlap
    # the likelihood batch's launch shape is tuned first, alone on the device
    cf.loglike_batch([problem], d_cl, [d_maps_scan], device=True, packed=[packed], autotune=True)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        parts(True, overlap)
        parts(False, overlap)
    torch.cuda.synchronize()
    reps, part_ms = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        # The last timed step carries per-stage device timers and an event pair around every GEMM
        # launch (the kernel timings of the roofline); the events cost about 6 ms of host time per
        # step, so the other steps run without them.
        timed = k == args.steps - 1
        (rq, tq), (rs, ts) = parts(timed, overlap)
        part_ms.append((1e3 * tq, 1e3 * ts))
        if timed:
            reps.append((rq, rs))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_tuned = _tuned_line(os.environ["CF_TUNE_CACHE"], n)     # the step's launch shape
    # each part alone: medians over steps run in sequence after the timed region (for the
    # overlapped step these are the parts' own times, which overlap inside the timed steps), and
    # one instrumented sequential step for the stage times and the whole factorisations' rates
    if overlap:
        seq_ms = [parts(False, False) for _ in range(max(3, min(args.steps, 10)))]
        qml_ms = [1e3 * q[1] for q, _ in seq_ms]
        scan_ms = [1e3 * l[1] for _, l in seq_ms]
        (sq, _), (sl, _) = parts(True, False)
        seq_rep = (sq, sl)
    else:
        plain = range(args.steps - 1) if args.steps > 1 else range(args.steps)
        qml_ms = [part_ms[k][0] for k in plain]
        scan_ms = [part_ms[k][1] for k in plain]
        seq_rep = reps[-1]
    ms_step = 1000.0 * wall / args.steps
    stage = np.asarray(seq_rep[0]["ms_stage"])
    scan_stage = np.asarray(seq_rep[1]["ms_stage"])

    def instances(rr):
        """GEMM instances over instrumented steps (both calls): event time, algorithmic flops,
        launches, sorted by device time."""
        g_ms = np.sum([np.add(r[0]["gemm_ms"], r[1]["gemm_ms"]) for r in rr], axis=0)
        g_fl = np.sum([np.add(r[0]["gemm_flops"], r[1]["gemm_flops"]) for r in rr], axis=0)
        g_n = np.sum([np.add(r[0]["gemm_launches"], r[1]["gemm_launches"]) for r in rr], axis=0)
        g_by = np.sum([np.add(r[0]["gemm_bytes"], r[1]["gemm_bytes"]) for r in rr], axis=0)
        res = []
        for i in range(len(g_ms)):
            if g_n[i] > 0:
                res.append({"kernel": cf.gemm_instance_name(i), "launches_per_step": float(g_n[i]) / len(rr),
                            "ms_per_step": float(g_ms[i]) / len(rr), "avg_launch_us": float(g_ms[i] / g_n[i]) * 1e3,
                            "tflops": float(g_fl[i] / (g_ms[i] * 1e-3) / 1e12) if g_ms[i] > 0 else None,
                            "flops_per_launch": float(g_fl[i] / g_n[i]),
                            "algorithmic_bytes_per_launch": float(g_by[i] / g_n[i])})
        res.sort(key=lambda r: -r["ms_per_step"])
        return res
    mixed = None if args.no_mixed else mixed_precision(cf, I, problem, bins, packed, d_maps_qml, d_cl,
                                                          d_maps_scan)
    extras = None if args.no_extras else qml_extras(cf, I, problem, bins, packed, d_maps_qml)
    scan_qu = None if args.no_extras else qu_scan(cf, I, args.scan_points)
    scan_tqu = None if args.no_extras else tqu_scan(cf, I, problem, packed, d_maps_scan)
    fishers = None if args.no_extras else other_fishers(cf, I)
    host_inputs = None if args.no_extras else host_input_step(cf, problem, bins, maps_qml, maps_scan,
                                                                 cl_points)
    smw = None
    if not args.no_smw:
        direct_m2 = cf.loglike_batch([problem], d_cl, [d_maps_scan], device=True, packed=[packed],
                                     autotune=True)["m2lnL"][:, 0, :].cpu().numpy()
        smw = smw_section(cf, I, problem, packed, d_maps_scan, direct_m2,
                          SCAN_POINTS / (np.median(scan_ms) * 1e-3))
    # Roofline kernel: the GEMM instance with the most device time in the instrumented timed step
    # (the Cholesky updates C -= L L^T of the two factorisations), achieved = its algorithmic flops
    # in that step / its summed HIP-event durations on the streams it ran on.  Every instance is
    # also listed (gemm_instances), with the whole factorisations' rates (factorisation).  With
    # the parts overlapped, each launch shares the device with the other part's kernels;
    # roofline_sequential gives the same instance in the instrumented sequential step.
    inst = instances(reps)
    top = inst[0]
    inst_seq = instances([seq_rep]) if overlap else inst
    top_seq = [r for r in inst_seq if r["kernel"] == top["kernel"]][0]
    traffic = _traffic(top["kernel"])
    # whole factorisations against the same peak, algorithmic flops only: n^3/3 for the Cholesky and
    # m^2 per right-hand side solved over m rows (the E,B columns of Y vanish above the first Q
    # pixel, so they are solved over n - p0 rows; the T columns and the map over all n)
    npx = problem.npix
    p0 = (npx // 64) * 64
    nT = 48 * 48 - 4
    fac_fisher = n ** 3 / 3.0 + (nT + 1) * n ** 2 + (6900 - nT) * (n - p0) ** 2
    fac_scan = SCAN_POINTS * (n ** 3 / 3.0 + NMAPS_SCAN * n ** 2)
    factorisation = {}
    for key, fl, ms in (("fisher", fac_fisher, stage[1]), ("loglike", fac_scan, scan_stage[1])):
        tf = fl / (ms * 1e-3) / 1e12
        factorisation[key] = {"flops": fl, "ms": round(float(ms), 4), "tflops": tf,
                              "frac": tf / PEAK_FP64_TFLOPS}
    out = {
        "metric": "Fisher wall time & −2lnL evals/s, FP64 vs mixed/emulator, Nside16 TQU",
        "value": 1000.0 / ms_step,
        "unit": "steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": ("TQU N_side 16, |b|>20 deg (n=5952), l 2-47, 6 spectra x 12 bins; "
                                f"step = Fisher+QML (1 map) + -2lnL at {SCAN_POINTS} points x "
                                f"{NMAPS_SCAN} maps"),
                   "precision": "fp64", "n": n, "nmodes": 6900, "scan_points_per_step": SCAN_POINTS,
                   "maps_per_point": NMAPS_SCAN,
                   "parts": "overlapped" if overlap else "sequential",
                   "autotuned": step_tuned},
        "fisher_qml_ms": float(np.median(qml_ms)),
        "loglike_ms": float(np.median(scan_ms)),
        "loglike_points_per_s": SCAN_POINTS / (np.median(scan_ms) * 1e-3),
        "loglike_map_evals_per_s": SCAN_POINTS * NMAPS_SCAN / (np.median(scan_ms) * 1e-3),
        "stages_fisher_qml_ms": dict(zip(cf.STAGES, [round(float(x), 4) for x in stage])),
        "stages_loglike_ms": dict(zip(cf.STAGES, [round(float(x), 4) for x in scan_stage])),
        "gemm_instances": inst,
        "mixed_precision": mixed,
        "smw": smw,
        "qml_extras": extras,
        "host_inputs": host_inputs,
        "qu_scan": scan_qu,
        "tqu_scan": scan_tqu,
        "other_fishers": fishers,
        "factorisation": factorisation,
        "roofline_sequential": {"kernel": top_seq["kernel"], "avg_launch_us": top_seq["avg_launch_us"],
                                "achieved": top_seq["tflops"], "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                "frac": top_seq["tflops"] / PEAK_FP64_TFLOPS,
                                "launches_per_step": top_seq["launches_per_step"],
                                "flops_per_launch": top_seq["flops_per_launch"]},
        "roofline": {"bound": "mfma", "kernel": top["kernel"] + " FP64 " + GEMM_ROLE.get(top["kernel"][-2], ""),
                     "avg_launch_us": top["avg_launch_us"],
                     "achieved": top["tflops"], "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": top["tflops"] / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "launches_per_step": top["launches_per_step"],
                     "flops_per_launch": top["flops_per_launch"],
                     "algorithmic_bytes_per_launch": top["algorithmic_bytes_per_launch"]},
    }
    if not args.no_emulator:
        out["emulator"] = emulator_bench(cf, I, args.emu_train, args.emu_epochs, args.emu_query)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problem, bins, cl_points, maps_qml, maps_scan,
                                           full=args.cpu_baseline_full)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
