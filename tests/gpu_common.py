"""Helpers shared by the GPU parity tests (metrics of the parity contract)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_np(x):
    if type(x).__module__.startswith("torch"):
        return x.detach().cpu().numpy()
    return np.asarray(x)


def metric_C(A, B):
    """max |dC_ij| / sqrt(C_ii C_jj)"""
    d = np.sqrt(np.abs(np.diag(B)))
    return float(np.max(np.abs(A - B) / np.outer(d, d)))


def metric_F(A, B):
    """max |dF_ij| / sqrt(F_ii F_jj)"""
    d = np.sqrt(np.abs(np.diag(B)))
    return float(np.max(np.abs(A - B) / np.outer(d, d)))


def metric_vec_fisher(a, b, F):
    """max_b |da_b| / sqrt(F_bb): shift in units of the estimator noise of q (Cov(q) = F)."""
    return float(np.max(np.abs(np.atleast_2d(a) - np.atleast_2d(b)) / np.sqrt(np.diag(F))[None, :]))


def metric_chat(a, b, F):
    """max_b |dChat_b| / sqrt((F^-1)_bb)."""
    s = np.sqrt(np.diag(np.linalg.inv(F)))
    return float(np.max(np.abs(np.atleast_2d(a) - np.atleast_2d(b)) / s[None, :]))
