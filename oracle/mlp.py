"""FP64 reference of the likelihood emulator: an MLP in -> w -> ... -> w -> 1 with SiLU, its
mean-squared-error gradient and one Adam step.

Oracle code: test infrastructure only (see oracle/__init__.py).

Parameters are a list [(W1, b1), ..., (WL, bL)] with W_l of shape [out][in] (y = x W^T + b).
With ``bf16=True`` the operands of the hidden-to-hidden products (layers 2..L-1: their weights and
their input activations) are rounded to bfloat16 (round-to-nearest-even), the precision in which
the GPU feeds those products to its matrix cores; the input and output layers stay unrounded.
This lets the GPU passes be compared with this one on equal operands.
"""
import numpy as np


def round_bf16(x):
    """Round float64 -> float32 -> bfloat16 (nearest even) and back to float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _hidden(l, nlayers):
    """Layer l (0-based) maps hidden to hidden: neither the first nor the last layer."""
    return 0 < l < nlayers - 1


def init_params(sizes, rng):
    """Uniform(-1/sqrt(in), 1/sqrt(in)) weights and biases (any fixed rule works for the checks)."""
    params = []
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        a = 1.0 / np.sqrt(fin)
        params.append((rng.uniform(-a, a, (fout, fin)), rng.uniform(-a, a, fout)))
    return params


def forward(params, x, bf16=False):
    """Returns the output [B] and the per-layer (input, pre-activation) cache."""
    h = np.asarray(x, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(params):
        q = bf16 and _hidden(l, len(params))
        hin = round_bf16(h) if q else h
        Wq = round_bf16(W) if q else W
        z = hin @ Wq.T + b
        cache.append((hin, z))
        h = silu(z) if l < len(params) - 1 else z
    return h[:, 0], cache


def loss_and_grads(params, x, y, bf16=False):
    """MSE = mean((f(x) - y)^2) and its gradients with respect to every W_l, b_l."""
    out, cache = forward(params, x, bf16)
    B = out.shape[0]
    r = out - y
    loss = np.mean(r * r)
    d = (2.0 / B) * r[:, None]                    # dL/dz of the last layer
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        hin, z = cache[l]
        W = params[l][0]
        Wq = round_bf16(W) if bf16 and _hidden(l, len(params)) else W
        grads[l] = (d.T @ hin, d.sum(axis=0))
        if l > 0:
            dh = d @ Wq
            d = dh * silu_grad(cache[l - 1][1])
    return loss, grads


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new params, m, v."""
    newp, newm, newv = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        out = []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = beta1 * mm + (1 - beta1) * g
            vv = beta2 * vv + (1 - beta2) * g * g
            mh = mm / (1 - beta1 ** t)
            vh = vv / (1 - beta2 ** t)
            out.append((p - lr * mh / (np.sqrt(vh) + eps), mm, vv))
        newp.append((out[0][0], out[1][0]))
        newm.append((out[0][1], out[1][1]))
        newv.append((out[0][2], out[1][2]))
    return newp, newm, newv
