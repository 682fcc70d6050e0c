"""GPU checks of the likelihood emulator (forward, gradient, Adam, training loop, prediction with
exact fallback) against the FP64 oracle MLP running the same bfloat16-rounded operands."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import mlp  # noqa: E402
from paper_2605_21149_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    _cf().lib()
    assert torch.cuda.is_available(), "GPU tests selected but torch sees no GPU"


def _cf():
    from paper_2605_21149_amd import cf
    return cf


def _layers(flat, in_dim, width, depth):
    """Split the flat FP32 parameter vector (W_l [out][in] then b_l, layer by layer) into the
    oracle's [(W, b), ...] in float64."""
    sizes = [in_dim] + [width] * depth + [1]
    out, o = [], 0
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        W = flat[o:o + fin * fout].astype(np.float64).reshape(fout, fin)
        o += fin * fout
        b = flat[o:o + fout].astype(np.float64)
        o += fout
        out.append((W, b))
    assert o == flat.size
    return out


def _flat(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


SHAPES = [(7, 64, 2, 2), (7, 256, 3, 1), (3, 128, 1, 1), (5, 128, 4, 2)]


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_oracle(shape):
    cf = _cf()
    in_dim, W, D, E = shape
    emu = cf.Emulator(in_dim, W, D, E, seed=11)
    rng = np.random.default_rng(12)
    x = rng.uniform(-1, 1, (203, in_dim))      # 3 full row tiles and a ragged one
    out = emu.forward(x)
    for e in range(E):
        ref, _ = mlp.forward(_layers(emu.get_params(e), in_dim, W, D), x, bf16=True)
        err = np.max(np.abs(out[e] - ref)) / max(1e-3, np.max(np.abs(ref)))
        print(f"forward {shape} member {e}: rel err {err:.2e}", flush=True)
        assert err <= 1e-2


@pytest.mark.parametrize("shape", SHAPES)
def test_gradient_matches_oracle(shape):
    cf = _cf()
    in_dim, W, D, E = shape
    emu = cf.Emulator(in_dim, W, D, E, seed=21)
    rng = np.random.default_rng(22)
    N = 200
    x = rng.uniform(-1, 1, (N, in_dim))
    y = np.sin(x.sum(axis=1)) + 0.1 * rng.standard_normal(N)
    g, loss = emu.gradient(x, y)
    for e in range(E):
        layers = _layers(emu.get_params(e), in_dim, W, D)
        l_ref, gr = mlp.loss_and_grads(layers, x, y, bf16=True)
        gref = _flat(gr)
        cos = float(g[e] @ gref / (np.linalg.norm(g[e]) * np.linalg.norm(gref)))
        rel = float(np.linalg.norm(g[e] - gref) / np.linalg.norm(gref))
        print(f"gradient {shape} member {e}: cos {cos:.7f} rel {rel:.2e} loss {loss[e]:.6f} vs {l_ref:.6f}",
              flush=True)
        assert cos >= 0.999 and rel <= 1e-2
        assert abs(loss[e] - l_ref) <= 1e-3 * abs(l_ref)


def test_adam_steps_match_oracle():
    cf = _cf()
    in_dim, W, D, E = 7, 64, 2, 2
    emu = cf.Emulator(in_dim, W, D, E, seed=31)
    rng = np.random.default_rng(32)
    p0 = [_layers(emu.get_params(e), in_dim, W, D) for e in range(E)]
    zeros = [[(np.zeros_like(Wl), np.zeros_like(bl)) for Wl, bl in p] for p in p0]
    m, v, p = zeros, [list(z) for z in zeros], p0
    for t, lr in ((1, 1e-3), (2, 5e-4)):
        g = rng.standard_normal((E, emu.P)).astype(np.float32) * np.float32(1e-2)
        emu.adam(g, lr)
        for e in range(E):
            ge = _layers(g[e], in_dim, W, D)
            newp, m_e, v_e = mlp.adam_step(p[e], ge, m[e], v[e], t, lr)
            got = emu.get_params(e).astype(np.float64)
            err = np.max(np.abs(got - _flat(newp)))
            print(f"adam t={t} member {e}: max |dp| {err:.2e}", flush=True)
            assert err <= 1e-6
            # continue the oracle from the GPU's FP32 parameters so that steps do not compound
            p[e] = _layers(emu.get_params(e), in_dim, W, D)
            m[e], v[e] = m_e, v_e


def test_train_step_equals_gradient_then_adam():
    """One fused training step (row kernel + weight-gradient kernel with Adam in its epilogue)
    lands where the separate gradient and Adam entry points land."""
    cf = _cf()
    in_dim, W, D = 7, 128, 3
    rng = np.random.default_rng(41)
    N = 256
    x = rng.uniform(0.5, 1.5, (N, in_dim))
    y = 100.0 + 20.0 * np.cos(x @ rng.uniform(-1, 1, in_dim))
    a = cf.Emulator(in_dim, W, D, 1, seed=42)
    b = cf.Emulator(in_dim, W, D, 1, seed=42)
    lr = 1e-3
    a.train(x, y, epochs=1, batch=N, lr=lr, val_frac=0.0, baseline=0)
    lo, hi = x.min(axis=0), x.max(axis=0)
    xn = (2 * x - lo - hi) / (hi - lo)
    yn = (y - y.mean()) / y.std()
    g, _ = b.gradient(xn, yn)
    b.adam(g, lr)
    pa, pb = a.get_params(0).astype(np.float64), b.get_params(0).astype(np.float64)
    d = np.abs(pa - pb)
    print(f"train step vs gradient+adam: max {d.max():.2e}, frac > 1e-6: {np.mean(d > 1e-6):.2e}", flush=True)
    # the two sum the batch rows in different orders; Adam's first step (about lr * sign(g)) only
    # differs where a gradient entry is within rounding of zero
    assert np.mean(d > 1e-6) < 1e-3
    assert d.max() <= 2.5 * lr


def test_save_load_roundtrip(tmp_path):
    cf = _cf()
    rng = np.random.default_rng(51)
    x = rng.uniform(0, 1, (512, 3))
    y = (x ** 2).sum(axis=1)
    emu = cf.Emulator(3, 64, 2, 2, seed=52)
    emu.train(x, y, epochs=2, batch=128)
    path = tmp_path / "emu.bin"
    emu.save(path)
    back = cf.Emulator.load(path)
    assert (back.in_dim, back.width, back.depth, back.ensemble) == (3, 64, 2, 2)
    for e in range(2):
        np.testing.assert_array_equal(back.get_params(e), emu.get_params(e))
    q = rng.uniform(0, 1, (100, 3))
    r1, r2 = emu.predict(q, spread_max=1e9), back.predict(q, spread_max=1e9)
    np.testing.assert_array_equal(r1["y"], r2["y"])
    # training continues from the stored moments and step count identically
    emu.train(x, y, epochs=1, batch=128)
    back.train(x, y, epochs=1, batch=128)
    np.testing.assert_array_equal(back.get_params(1), emu.get_params(1))


def test_training_learns_a_smooth_function_and_routes_queries():
    cf = _cf()
    rng = np.random.default_rng(61)
    N = 20000
    A = rng.standard_normal((7, 7))
    A = A @ A.T / 7

    def f(t):
        u = t - 1.0
        return 3000.0 + 40.0 * np.einsum("ni,ij,nj->n", u, A, u) + 25.0 * np.sin(2 * u[:, 0]) - 30.0 * u[:, 6]

    x = rng.uniform(0.5, 1.5, (N, 7))
    emu = cf.Emulator(7, 256, 3, 4, seed=62)
    rep = emu.train(x, f(x), epochs=150, batch=1024, report=True)
    sig = f(x).std()
    print(f"train: {rep['ms_total']:.0f} ms, loss {rep['est_err'][0]:.2e}, held-out rms {rep['est_err'][1]:.3f}"
          f" max {rep['est_err'][2]:.3f} spread {rep['est_err'][3]:.3f} (sigma {sig:.1f})", flush=True)
    assert rep["est_err"][1] < 0.02 * sig
    q_in = rng.uniform(0.55, 1.45, (900, 7))
    q_out = rng.uniform(0.4, 1.6, (100, 7))
    q_out[:, 0] = np.where(rng.uniform(size=100) < 0.5, 0.45, 1.55)   # certainly outside the box
    q = np.concatenate([q_in, q_out])
    r = emu.predict(q, spread_max=0.1)
    assert np.all(r["fallback"][900:] == 1)
    inside_ok = r["fallback"][:900] == 0
    err = np.abs(r["y"][:900] - f(q_in))
    print(f"predict: fallback inside {1 - inside_ok.mean():.3f}, |err| p50 {np.median(err):.3f}"
          f" p99 {np.quantile(err, 0.99):.3f}", flush=True)
    assert np.all(r["spread"] >= 0)
    assert np.all((r["spread"][:900] > 0.1) == ~inside_ok)
    assert np.median(err) < 0.02 * sig


def test_prediction_falls_back_to_the_exact_likelihood():
    """Queries outside the hull (or too uncertain) get the exact FP64 -2lnL of cf_loglike_batch."""
    cf = _cf()
    p = I.qu_scan_problem(8)
    L = p.lmax + 1
    base = I.scan_spectra(np.zeros((1, 7)), p.cl)[0]
    basis = np.stack([I.scan_spectra(np.eye(7)[k:k + 1], p.cl)[0] - base for k in range(7)])
    dmap = I.white_maps(p.n, 1, seed=402)[0]
    xt = I.scan_points(256, seed=501)
    cl_t = base[None] + np.einsum("nk,kxl->nxl", xt, basis)
    exact_t = cf.loglike_batch([p], cl_t[:, None], [dmap[None]])["m2lnL"][:, 0, 0]
    emu = cf.Emulator(7, 64, 2, 2, seed=503)
    emu.train(xt, exact_t, epochs=20, batch=64, val_frac=0.0)
    q = np.concatenate([I.scan_points(24, seed=506), I.scan_points(8, seed=507, lo=1.55, hi=1.6)])
    r = emu.predict(q, spread_max=0.5, exact=(p, base, basis, dmap))
    cl_q = base[None] + np.einsum("nk,kxl->nxl", q, basis)
    exact_q = cf.loglike_batch([p], cl_q[:, None], [dmap[None]])["m2lnL"][:, 0, 0]
    fb = r["fallback"].astype(bool)
    assert fb[24:].all()
    np.testing.assert_allclose(r["y"][fb], exact_q[fb], rtol=1e-12)
    print(f"fallback {fb.sum()} of {fb.size}; emulated |err| max "
          f"{np.max(np.abs(r['y'][~fb] - exact_q[~fb])) if (~fb).any() else 0:.3f}", flush=True)
    # with the fallback disabled the same queries are only flagged
    r2 = emu.predict(q, spread_max=0.5)
    np.testing.assert_array_equal(r2["fallback"], r["fallback"])
    np.testing.assert_array_equal(r2["y"][~fb], r["y"][~fb])


def test_quadratic_baseline_carries_a_quadratic_target():
    """With the degree-2 baseline a (nearly) quadratic target is reproduced by the least-squares
    fit alone; the networks only see the tiny residual."""
    cf = _cf()
    rng = np.random.default_rng(71)
    x = rng.uniform(0.5, 1.5, (4096, 7))
    B = rng.standard_normal((7, 7))
    c = rng.standard_normal(7)

    def f(t):
        return 500.0 + t @ c * 30.0 + 10.0 * np.einsum("ni,ij,nj->n", t, B, t) + 1e-6 * np.sin(5 * t[:, 0])

    emu = cf.Emulator(7, 64, 2, 2, seed=72)
    emu.train(x, f(x), epochs=2, batch=512, baseline=2)
    q = rng.uniform(0.5, 1.5, (500, 7))
    err = np.max(np.abs(emu.predict(q, spread_max=1e9)["y"] - f(q)))
    print(f"quadratic target: max |err| {err:.2e} (sigma {f(x).std():.1f})", flush=True)
    assert err <= 1e-4 * f(x).std()


@pytest.mark.timeout(900)
def test_emulator_gain_over_the_fastest_exact_path():
    """The QU N_side 16 scan problem (n = 3968), one map, 7 parameters (6 EE band amplitudes over
    l 2..29 and the reionisation bump) whose spectra vary only inside the E window l 2..29.  The
    fastest exact likelihood of the library there is the harmonic-basis handle of that window
    (cf_smw_loglike, one 896-mode factorisation per point).  The 4-member ensemble is trained on
    65536 of its evaluations; on 16384 queries (90 % in the parameter box, 10 % from [0.4, 1.6]^7)
    with the exact fallback through the same handle, the emulated values are within 0.1 of the exact
    ones at the 99th percentile, and queries are answered (fallback included) faster than the handle
    answers them alone."""
    import time
    import torch
    cf = _cf()
    p = I.qu_scan_problem(16)
    dmap = torch.as_tensor(I.white_maps(p.n, 1, 403, rms=3.0)).cuda()
    base = I.scan_spectra(np.zeros((1, 7)), p.cl)[0]
    basis = np.stack([I.scan_spectra(np.eye(7)[k:k + 1], p.cl)[0] - base for k in range(7)])

    def spectra(x):
        return torch.as_tensor(np.ascontiguousarray(base[None] + np.einsum("nk,kxl->nxl", x, basis))).cuda()

    with cf.SMW(p, dmap, (2, 29), "E", device=True) as h:
        xt = I.scan_points(65536, seed=511)
        yt = torch.cat([h.loglike(spectra(xt[i:i + 16384]))["m2lnL"][:, 0] for i in range(0, 65536, 16384)])
        emu = cf.Emulator(7, 256, 3, 4, seed=512)
        tr = emu.train(torch.as_tensor(xt).cuda(), yt, epochs=100, batch=1024, device=True, report=True)
        print(f"trained: {tr['ir_iters']} steps, held-out rms {tr['est_err'][1]:.4f}", flush=True)
        q = np.concatenate([I.scan_points(14746, seed=513), I.scan_points(1638, seed=514, lo=0.4, hi=1.6)])
        d_q = torch.as_tensor(q).cuda()
        cl_q = spectra(q)
        h.loglike(cl_q[:512])
        emu.predict(d_q[:1024], spread_max=0.1, device=True, exact_smw=(h, base, basis))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        exact = h.loglike(cl_q)["m2lnL"][:, 0]
        torch.cuda.synchronize()
        t_exact = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = emu.predict(d_q, spread_max=0.1, device=True, exact_smw=(h, base, basis))
        torch.cuda.synchronize()
        t_emu = time.perf_counter() - t0
    fb = r["fallback"].cpu().numpy().astype(bool)
    err = np.abs(r["y"].cpu().numpy() - exact.cpu().numpy())
    p99 = float(np.quantile(err[~fb], 0.99))
    rate_exact, rate_emu = len(q) / t_exact, len(q) / t_emu
    print(f"fallback {fb.mean():.3f}, emulated |d(-2lnL)| p50 {np.median(err[~fb]):.4f} p99 {p99:.4f} "
          f"max {err[~fb].max():.4f}; fallback max {err[fb].max() if fb.any() else 0.0:.2e}; "
          f"exact {rate_exact:.0f}/s, emulator with fallback {rate_emu:.0f}/s ({rate_emu / rate_exact:.1f}x)",
          flush=True)
    assert p99 <= 0.1
    assert (not fb.any()) or err[fb].max() < 1e-9          # the fallback values are the exact ones
    assert rate_emu > rate_exact
