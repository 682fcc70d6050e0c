"""ctypes binding of libcf (include/cf.h): argument marshalling only.

Every function here packs numpy arrays (host memory) or torch CUDA tensors (device memory)
into the C structs of cf.h and calls the library; all arithmetic of the path runs in the
library's HIP kernels.  Loading fails loudly when libcf.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcf.so")

CF_OK, CF_EINVAL, CF_ENOTPD, CF_ENOMEM, CF_EDEVICE, CF_ENOCONV = range(6)
CF_FP64, CF_MIXED_FP32, CF_MIXED_BF16X3 = 0, 1, 2
FIELDS = {"T": 1, "QU": 2, "TQU": 3}
SPEC_BITS = {"TT": 1, "EE": 2, "BB": 4, "TE": 8, "TB": 16, "EB": 32}
CF_NOISE_DIAG, CF_NOISE_DENSE = 0, 1
CF_MEM_HOST, CF_MEM_DEVICE = 0, 1
_STATUS = {1: "CF_EINVAL", 2: "CF_ENOTPD", 3: "CF_ENOMEM", 4: "CF_EDEVICE", 5: "CF_ENOCONV"}

_dp = C.POINTER(C.c_double)


class cf_problem(C.Structure):
    _fields_ = [("nside", C.c_int32), ("mask", C.POINTER(C.c_uint8)), ("ndir", C.c_int64),
                ("theta", _dp), ("phi", _dp), ("fields", C.c_int32), ("lmin", C.c_int32),
                ("lmax", C.c_int32), ("cl", _dp), ("bl", _dp), ("pl", _dp),
                ("noise_kind", C.c_int32), ("noise", _dp), ("noise_rank", C.c_int32),
                ("noise_U", _dp), ("mem", C.c_int32)]


class cf_bins(C.Structure):
    _fields_ = [("nbins", C.c_int32), ("lo", C.POINTER(C.c_int32)), ("hi", C.POINTER(C.c_int32)),
                ("spectra", C.c_uint32)]


class cf_exec(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("stage_timing", C.c_int32), ("refine_max", C.c_int32),
                ("allow_fallback", C.c_int32), ("no_graph", C.c_int32), ("autotune", C.c_int32)]


class cf_report(C.Structure):
    _fields_ = [("ms_total", C.c_double), ("ms_stage", C.c_double * 8), ("flops", C.c_double),
                ("logdet", C.c_double), ("n", C.c_int64), ("nmodes", C.c_int64),
                ("fail_index", C.c_int32), ("ir_iters", C.c_int32), ("est_err", C.c_double * 4),
                ("n_fallback", C.c_int64), ("gemm_ms", C.c_double * 16), ("gemm_flops", C.c_double * 16),
                ("gemm_launches", C.c_int64 * 16), ("gemm_bytes", C.c_double * 16)]

    def as_dict(self):
        return {"ms_total": self.ms_total, "ms_stage": list(self.ms_stage), "flops": self.flops,
                "logdet": self.logdet, "n": self.n, "nmodes": self.nmodes,
                "fail_index": self.fail_index, "ir_iters": self.ir_iters,
                "est_err": list(self.est_err), "n_fallback": self.n_fallback,
                "gemm_ms": list(self.gemm_ms), "gemm_flops": list(self.gemm_flops),
                "gemm_launches": list(self.gemm_launches), "gemm_bytes": list(self.gemm_bytes)}


def gemm_instance_name(i):
    """Kernel name of FP64 GEMM instance id i of cf_report.gemm_* (tile, operand storage, tag):
    ids 0-7 untagged (bit 0: 128 tile, bit 1: A transposed, bit 2: B transposed); 8-9 the
    Z = G^T G product, 10-11 the Cholesky updates (bit 0: 128 tile; A plain, B transposed)."""
    t = 128 if i & 1 else 64
    if i >= 8:
        return f"k_gemm<{t}, {t}, false, true, {1 + (i - 8) // 2}>"
    return f"k_gemm<{t}, {t}, {'true' if i & 2 else 'false'}, {'true' if i & 4 else 'false'}, 0>"


STAGES = ("build", "potrf", "ybuild", "trsm", "syrk", "reduce", "qml", "other")

# Every symbol include/cf.h declares.
EXPORTS = ("cf_problem_dim", "cf_problem_nmodes", "cf_cov_build", "cf_fisher", "cf_qml",
           "cf_loglike_batch", "cf_loglike_batch_noalloc", "cf_emu_create", "cf_emu_destroy", "cf_emu_param_count", "cf_emu_shape",
           "cf_emu_train", "cf_emu_predict", "cf_emu_predict_smw", "cf_emu_get_params", "cf_emu_set_params",
           "cf_emu_forward", "cf_emu_gradient", "cf_emu_adam", "cf_emu_save", "cf_emu_load",
           "cf_smw_create", "cf_smw_loglike", "cf_smw_dim", "cf_smw_destroy", "cf_select_basis", "cf_loglike_auto", "cf_smw_qml", "cf_qml_joint", "cf_decorrelate", "cf_qml_iterate", "cf_qml_cross",
           "cf_last_error", "cf_version")


class cf_basis_choice(C.Structure):
    _fields_ = [("basis", C.c_int32), ("harmonic_ok", C.c_int32), ("groups", C.c_int32), ("n", C.c_int64),
                ("k_win", C.c_int64), ("cost_pixel", C.c_double), ("cost_harmonic", C.c_double)]

    def as_dict(self):
        return {"basis": "harmonic" if self.basis else "pixel", "harmonic_ok": bool(self.harmonic_ok),
                "groups": self.groups, "n": self.n, "k_win": self.k_win, "cost_pixel": self.cost_pixel,
                "cost_harmonic": self.cost_harmonic}


class cf_linear_spectra(C.Structure):
    _fields_ = [("nparam", C.c_int32), ("lstride", C.c_int32), ("base", _dp), ("basis", _dp)]


class cf_emu_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("val_frac", C.c_double), ("baseline", C.c_int32)]


class CFError(RuntimeError):
    def __init__(self, status, msg, report=None):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status
        self.report = report


_lib = None


def lib():
    """Load libcf.so (raises when it has not been built: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2605_21149_amd/build.py")
        # torch ships its own HIP runtime; loading it first makes libcf bind to that same runtime
        # (one runtime per process), whichever of the two the caller touches first.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        L.cf_last_error.restype = C.c_char_p
        L.cf_version.restype = C.c_char_p
        L.cf_problem_dim.restype = C.c_int64
        L.cf_problem_dim.argtypes = [C.POINTER(cf_problem)]
        L.cf_problem_nmodes.restype = C.c_int64
        L.cf_problem_nmodes.argtypes = [C.POINTER(cf_problem)]
        L.cf_cov_build.argtypes = [C.POINTER(cf_problem), _dp, C.POINTER(C.c_int64),
                                   C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_fisher.argtypes = [C.POINTER(cf_problem), C.POINTER(cf_bins), C.c_int32, _dp,
                                C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_qml.argtypes = [C.POINTER(cf_problem), C.POINTER(cf_bins), _dp, C.c_int32, C.c_int32,
                             _dp, _dp, _dp, _dp, C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_loglike_batch.argtypes = [C.POINTER(cf_problem), C.c_int32, C.c_int32, _dp, C.c_int32,
                                       C.POINTER(_dp), C.c_int32, C.c_int32, _dp, _dp, _dp,
                                       C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_loglike_batch_noalloc.argtypes = L.cf_loglike_batch.argtypes
        _fp = C.POINTER(C.c_float)
        L.cf_emu_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                    C.POINTER(C.c_void_p)]
        L.cf_emu_destroy.argtypes = [C.c_void_p]
        L.cf_emu_destroy.restype = None
        L.cf_emu_param_count.argtypes = [C.c_void_p]
        L.cf_emu_param_count.restype = C.c_int64
        _ip = C.POINTER(C.c_int32)
        L.cf_emu_shape.argtypes = [C.c_void_p, _ip, _ip, _ip, _ip]
        L.cf_emu_train.argtypes = [C.c_void_p, _dp, _dp, C.c_int64, C.c_int32,
                                   C.POINTER(cf_emu_opts), C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_emu_predict.argtypes = [C.c_void_p, _dp, C.c_int64, C.c_int32, C.c_double,
                                     C.POINTER(cf_problem), C.POINTER(cf_linear_spectra), _dp, _dp,
                                     _dp, C.POINTER(C.c_uint8), C.POINTER(cf_exec),
                                     C.POINTER(cf_report)]
        L.cf_emu_predict_smw.argtypes = [C.c_void_p, _dp, C.c_int64, C.c_int32, C.c_double, C.c_void_p,
                                         C.POINTER(cf_linear_spectra), _dp, _dp, C.POINTER(C.c_uint8),
                                         C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_emu_get_params.argtypes = [C.c_void_p, C.c_int32, _fp]
        L.cf_emu_set_params.argtypes = [C.c_void_p, C.c_int32, _fp]
        L.cf_emu_forward.argtypes = [C.c_void_p, _dp, C.c_int64, _fp]
        L.cf_emu_gradient.argtypes = [C.c_void_p, _dp, _dp, C.c_int64, _fp, _dp]
        L.cf_emu_adam.argtypes = [C.c_void_p, _fp, C.c_double]
        L.cf_emu_save.argtypes = [C.c_void_p, C.c_char_p]
        L.cf_emu_load.argtypes = [C.c_char_p, C.POINTER(C.c_void_p)]
        L.cf_smw_create.argtypes = [C.POINTER(cf_problem), C.c_int32, C.c_int32, C.c_uint32, _dp, C.c_int32,
                                    C.POINTER(cf_exec), C.POINTER(C.c_void_p), C.POINTER(cf_report)]
        L.cf_smw_loglike.argtypes = [C.c_void_p, C.c_int32, _dp, C.c_int32, _dp, _dp, _dp,
                                     C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_qml_cross.argtypes = [C.POINTER(cf_problem), C.POINTER(cf_problem), C.POINTER(cf_bins), _dp, _dp,
                                   C.c_int32, _dp, _dp, _dp, C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_decorrelate.argtypes = [_dp, C.c_int32, _dp, C.c_int32, C.c_int32, _dp, _dp,
                                     C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_qml_iterate.argtypes = [C.POINTER(cf_problem), C.POINTER(cf_bins), _dp, C.c_int32, C.c_double,
                                     _dp, _dp, _dp, C.POINTER(C.c_int32), C.POINTER(cf_exec),
                                     C.POINTER(cf_report)]
        L.cf_select_basis.argtypes = [C.POINTER(cf_problem), C.c_int32, C.c_int32, C.c_uint32, C.c_int32, C.c_int32,
                                      C.POINTER(cf_basis_choice)]
        L.cf_select_basis.restype = C.c_int
        L.cf_loglike_auto.argtypes = [C.POINTER(cf_problem), C.c_int32, C.c_int32, C.c_uint32, C.c_int32, _dp,
                                      C.c_int32, _dp, C.c_int32, _dp, _dp, _dp, C.POINTER(cf_basis_choice),
                                      C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_loglike_auto.restype = C.c_int
        L.cf_smw_qml.argtypes = [C.POINTER(cf_problem), C.c_int32, C.c_int32, C.POINTER(cf_bins), _dp, C.c_int32,
                                 _dp, _dp, _dp, _dp, C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_smw_qml.restype = C.c_int
        L.cf_qml_joint.argtypes = [C.POINTER(cf_problem), C.POINTER(cf_problem), _dp, C.POINTER(cf_bins), _dp, _dp,
                                   C.c_int32, _dp, _dp, _dp, _dp, C.POINTER(cf_exec), C.POINTER(cf_report)]
        L.cf_qml_joint.restype = C.c_int
        L.cf_smw_dim.argtypes = [C.c_void_p]
        L.cf_smw_dim.restype = C.c_int64
        L.cf_smw_destroy.argtypes = [C.c_void_p]
        L.cf_smw_destroy.restype = None
        for name in ("cf_cov_build", "cf_fisher", "cf_qml", "cf_loglike_batch", "cf_loglike_batch_noalloc",
                     "cf_emu_create",
                     "cf_emu_train", "cf_emu_predict", "cf_emu_predict_smw", "cf_emu_get_params", "cf_emu_set_params",
                     "cf_emu_forward", "cf_emu_gradient", "cf_emu_adam", "cf_emu_save",
                     "cf_emu_load", "cf_smw_create", "cf_smw_loglike", "cf_decorrelate", "cf_qml_cross",
                     "cf_qml_iterate"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().cf_last_error().decode()


# ------------------------------------------------------------------------------ marshalling
def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x, ctype=C.c_double):
    if x is None:
        return None
    if _is_torch(x):
        return C.cast(C.c_void_p(x.data_ptr()), C.POINTER(ctype))
    return x.ctypes.data_as(C.POINTER(ctype))


def _host(a, dtype=np.float64):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


@dataclass
class _Packed:
    struct: cf_problem
    keep: list


def pack_problem(p, device=False, torch_device="cuda") -> _Packed:
    """Build a cf_problem from an ``inputs.Problem``.  device=True stages the noise arrays as
    torch tensors on the GPU (mem = CF_MEM_DEVICE); otherwise they stay numpy host arrays."""
    keep = []
    s = cf_problem()
    s.nside = int(p.nside)
    if p.nside:
        if p.mask is not None:
            m = _host(p.mask, np.uint8)
            keep.append(m)
            s.mask = _ptr(m, C.c_uint8)
    else:
        th, ph = _host(p.theta), _host(p.phi)
        keep += [th, ph]
        s.ndir = th.shape[0]
        s.theta, s.phi = _ptr(th), _ptr(ph)
    s.fields = FIELDS[p.fields]
    s.lmin, s.lmax = int(p.lmin), int(p.lmax)
    cl, bl, pl = _host(p.cl), _host(p.bl), _host(p.pl)
    keep += [cl, bl, pl]
    s.cl, s.bl, s.pl = _ptr(cl), _ptr(bl), _ptr(pl)
    if p.noise_dense is not None:
        s.noise_kind = CF_NOISE_DENSE
        noise = p.noise_dense
        U = None
    else:
        s.noise_kind = CF_NOISE_DIAG
        noise = p.noise_diag
        U = p.noise_U
    noise = _to_mem(noise, device, torch_device)
    keep.append(noise)
    s.noise = _ptr(noise)
    if U is not None:
        U = _to_mem(U, device, torch_device)
        keep.append(U)
        s.noise_rank = U.shape[1]
        s.noise_U = _ptr(U)
    s.mem = CF_MEM_DEVICE if device else CF_MEM_HOST
    return _Packed(s, keep)


def _to_mem(a, device, torch_device):
    if device:
        import torch
        if _is_torch(a):
            return a.to(device=torch_device, dtype=torch.float64).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(torch_device)
    if _is_torch(a):
        raise TypeError("host call given a torch tensor")
    return _host(a)


def pack_bins(b):
    lo, hi = _host(b.lo, np.int32), _host(b.hi, np.int32)
    s = cf_bins()
    s.nbins = lo.shape[0]
    s.lo, s.hi = _ptr(lo, C.c_int32), _ptr(hi, C.c_int32)
    s.spectra = sum(SPEC_BITS[x] for x in b.spectra)
    return s, [lo, hi]


def _exec(stream=None, stage_timing=False, no_graph=False, autotune=False, refine_max=-1):
    e = cf_exec()
    e.stream = stream
    e.stage_timing = 1 if stage_timing else 0
    e.refine_max = refine_max
    e.allow_fallback = 0
    e.no_graph = 1 if no_graph else 0
    e.autotune = 1 if autotune else 0
    return e


def _torch_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(st, rep=None):
    if st != CF_OK:
        raise CFError(st, last_error(), rep.as_dict() if rep is not None else None)


def _alloc(shape, device):
    if device:
        import torch
        return torch.empty(shape, dtype=torch.float64, device="cuda")
    return np.empty(shape, dtype=np.float64)


# ------------------------------------------------------------------------------ entry points
def problem_dim(p) -> int:
    pk = pack_problem(p)
    return int(lib().cf_problem_dim(C.byref(pk.struct)))


def problem_nmodes(p) -> int:
    pk = pack_problem(p)
    return int(lib().cf_problem_nmodes(C.byref(pk.struct)))


def cov_build(p, device=False, stage_timing=False, report=False):
    """C = S + N as an [n][n] array (numpy, or a torch CUDA tensor when device=True)."""
    pk = pack_problem(p, device)
    n = int(lib().cf_problem_dim(C.byref(pk.struct)))
    _check(0 if n > 0 else CF_EINVAL)
    out = _alloc((n, n), device)
    rep = cf_report()
    ex = _exec(_torch_stream() if device else None, stage_timing)
    n_out = C.c_int64(0)
    st = lib().cf_cov_build(C.byref(pk.struct), _ptr(out), C.byref(n_out), C.byref(ex), C.byref(rep))
    _check(st, rep)
    return (out, rep.as_dict()) if report else out


def fisher(p, bins, precision=CF_FP64, device=False, stage_timing=False, report=False, packed=None):
    pk = packed or pack_problem(p, device)
    bs, keep = pack_bins(bins)
    K = len(bins.spectra) * bs.nbins
    out = _alloc((K, K), device)
    rep = cf_report()
    ex = _exec(_torch_stream() if device else None, stage_timing)
    st = lib().cf_fisher(C.byref(pk.struct), C.byref(bs), int(precision), _ptr(out), C.byref(ex),
                         C.byref(rep))
    _check(st, rep)
    return (out, rep.as_dict()) if report else out


def qml(p, bins, maps, precision=CF_FP64, device=False, stage_timing=False, report=False,
        packed=None):
    """Returns dict(y, bias, chat, F) for maps [nmaps][n]."""
    pk = packed or pack_problem(p, device)
    bs, keep = pack_bins(bins)
    K = len(bins.spectra) * bs.nbins
    if device:
        import torch
        mp = maps if _is_torch(maps) else torch.as_tensor(np.ascontiguousarray(maps, np.float64))
        mp = mp.to("cuda", torch.float64).contiguous()
        if mp.dim() == 1:
            mp = mp[None]
    else:
        mp = np.atleast_2d(_host(maps))
    nmaps = mp.shape[0]
    y, b, ch, F = _alloc((nmaps, K), device), _alloc((K,), device), _alloc((nmaps, K), device), \
        _alloc((K, K), device)
    rep = cf_report()
    ex = _exec(_torch_stream() if device else None, stage_timing)
    st = lib().cf_qml(C.byref(pk.struct), C.byref(bs), _ptr(mp), nmaps, int(precision), _ptr(y),
                      _ptr(b), _ptr(ch), _ptr(F), C.byref(ex), C.byref(rep))
    _check(st, rep)
    out = {"y": y, "bias": b, "chat": ch, "F": F}
    return (out, rep.as_dict()) if report else out


def qml_cross(p1, p2, bins, maps1, maps2, device=False, stage_timing=False, report=False,
              packed=None):
    """Cross-QML of two data sets (same model, different noise): dict(q, chat, W)."""
    pk1, pk2 = packed or (pack_problem(p1, device), pack_problem(p2, device))
    bs, keep = pack_bins(bins)
    K = len(bins.spectra) * bs.nbins

    def _maps(m):
        if device:
            import torch
            t = m if _is_torch(m) else torch.as_tensor(np.ascontiguousarray(m, np.float64))
            return torch.atleast_2d(t.to("cuda", torch.float64)).contiguous()
        return np.atleast_2d(_host(m))
    m1, m2 = _maps(maps1), _maps(maps2)
    nmaps = int(m1.shape[0])
    assert m2.shape[0] == nmaps
    q, ch, W = _alloc((nmaps, K), device), _alloc((nmaps, K), device), _alloc((K, K), device)
    rep = cf_report()
    ex = _exec(_torch_stream() if device else None, stage_timing)
    st = lib().cf_qml_cross(C.byref(pk1.struct), C.byref(pk2.struct), C.byref(bs), _ptr(m1), _ptr(m2), nmaps,
                            _ptr(q), _ptr(ch), _ptr(W), C.byref(ex), C.byref(rep))
    _check(st, rep)
    out = {"q": q, "chat": ch, "W": W}
    return (out, rep.as_dict()) if report else out


def loglike_batch(problems: Sequence, cl_points, maps: Sequence, precision=CF_FP64, device=False,
                  stage_timing=False, report=False, packed=None, no_graph=False, autotune=False, out=None,
                  noalloc=False):
    """-2 ln L over a scan.  cl_points [npoints][nprob][6][lstride]; maps[p] [nmaps][n_p].
    Returns dict(m2lnL [npoints][nprob][nmaps], chi2 (same), logdet [npoints][nprob]); out: optional
    caller-owned (m2lnL, chi2, logdet) arrays of those shapes to write into.  noalloc: call
    cf_loglike_batch_noalloc (the library's static scratch array; nothing is allocated by the
    library, the output arrays are the caller's or allocated here by the binding)."""
    pks = packed or [pack_problem(p, device) for p in problems]
    nprob = len(pks)
    arr = (cf_problem * nprob)(*[pk.struct for pk in pks])
    if device:
        import torch
        clp = cl_points if _is_torch(cl_points) else torch.as_tensor(np.ascontiguousarray(cl_points, np.float64))
        clp = clp.to("cuda", torch.float64).contiguous()
        mps = [(m if _is_torch(m) else torch.as_tensor(np.ascontiguousarray(m, np.float64))).to("cuda", torch.float64).contiguous() for m in maps]
    else:
        clp = _host(cl_points)
        mps = [np.atleast_2d(_host(m)) for m in maps]
    npoints, lstride = clp.shape[0], clp.shape[-1]
    assert clp.shape[1] == nprob and clp.shape[2] == 6
    nmaps = mps[0].shape[0]
    mptr = (_dp * nprob)(*[_ptr(m) for m in mps])
    if out is not None:
        m2, x2, ld = out
        assert tuple(m2.shape) == (npoints, nprob, nmaps) and tuple(ld.shape) == (npoints, nprob)
    else:
        m2 = _alloc((npoints, nprob, nmaps), device)
        x2 = _alloc((npoints, nprob, nmaps), device)
        ld = _alloc((npoints, nprob), device)
    rep = cf_report()
    ex = _exec(_torch_stream() if device else None, stage_timing, no_graph, autotune)
    fn = lib().cf_loglike_batch_noalloc if noalloc else lib().cf_loglike_batch
    st = fn(arr, nprob, npoints, _ptr(clp), lstride, mptr, nmaps, int(precision),
            _ptr(m2), _ptr(x2), _ptr(ld), C.byref(ex), C.byref(rep))
    _check(st, rep)
    out = {"m2lnL": m2, "chi2": x2, "logdet": ld}
    return (out, rep.as_dict()) if report else out


def qml_joint(p1, p2, bins, maps1, maps2, N12=None, device=False, report=False, packed=None):
    """Joint QML of two data sets of one sky (cf_qml_joint): p1 gives geometry, spectra and noise
    N1, p2 the noise N2; N12 [n][n] the shared noise (None: independent).  dict(y, bias, chat, F)."""
    pk1, pk2 = packed or (pack_problem(p1, device), pack_problem(p2, device))
    bs, keep = pack_bins(bins)
    K = len(bins.spectra) * bs.nbins

    def _dev(a):
        if device:
            import torch
            t = a if _is_torch(a) else torch.as_tensor(np.ascontiguousarray(a, np.float64))
            return t.to("cuda", torch.float64).contiguous()
        return np.ascontiguousarray(_host(a))
    m1 = _dev(maps1)
    m2 = _dev(maps2)
    if m1.ndim == 1:
        m1, m2 = m1[None], m2[None]
    x12 = None if N12 is None else _dev(N12)
    nm = int(m1.shape[0])
    y, bias, chat, F = (_alloc((nm, K), device), _alloc((K,), device), _alloc((nm, K), device),
                        _alloc((K, K), device))
    rep = cf_report()
    ex = _exec(_torch_stream() if device else None)
    st = lib().cf_qml_joint(C.byref(pk1.struct), C.byref(pk2.struct), _ptr(x12) if x12 is not None else None,
                            C.byref(bs), _ptr(m1), _ptr(m2), nm, _ptr(y), _ptr(bias), _ptr(chat), _ptr(F),
                            C.byref(ex), C.byref(rep))
    _check(st, rep)
    out = {"y": y, "bias": bias, "chat": chat, "F": F}
    return (out, rep.as_dict()) if report else out


def smw_qml(p, window, bins, maps, device=False, report=False, packed=None):
    """Fisher and QML in the harmonic basis with multipole switching (cf_smw_qml): the estimation
    window = (lo, hi) on every field of the problem, bins inside it.  Returns dict(y, bias, chat, F)."""
    pk = packed or pack_problem(p, device)
    bs, keep = pack_bins(bins)
    K = len(bins.spectra) * bs.nbins
    if device:
        import torch
        m = maps if _is_torch(maps) else torch.as_tensor(np.ascontiguousarray(maps, np.float64))
        m = torch.atleast_2d(m.to("cuda", torch.float64)).contiguous()
    else:
        m = np.atleast_2d(_host(maps))
    nm = int(m.shape[0])
    y, bias, chat, F = (_alloc((nm, K), device), _alloc((K,), device), _alloc((nm, K), device),
                        _alloc((K, K), device))
    rep = cf_report()
    ex = _exec(_torch_stream() if device else None)
    st = lib().cf_smw_qml(C.byref(pk.struct), int(window[0]), int(window[1]), C.byref(bs), _ptr(m), nm, _ptr(y),
                          _ptr(bias), _ptr(chat), _ptr(F), C.byref(ex), C.byref(rep))
    _check(st, rep)
    out = {"y": y, "bias": bias, "chat": chat, "F": F}
    return (out, rep.as_dict()) if report else out


def _field_bits(fields):
    return sum(FIELD_BITS[f] for f in set(fields))


def select_basis(p, window, fields, npoints, nmaps, packed=None):
    """The cost-based basis choice (cf_select_basis) for a scan of npoints points and nmaps maps
    whose spectra vary in window = (lo, hi) on the harmonic fields `fields` (e.g. "TEB")."""
    pk = packed or pack_problem(p)
    out = cf_basis_choice()
    _check(lib().cf_select_basis(C.byref(pk.struct), int(window[0]), int(window[1]), _field_bits(fields),
                                 int(npoints), int(nmaps), C.byref(out)))
    return out.as_dict()


def loglike_auto(p, window, fields, cl_points, maps, device=False, packed=None, report=False):
    """-2 ln L of one problem over cl_points [npoints][6][lstride] in the basis cf_select_basis picks
    (cf_loglike_auto).  Returns dict(m2lnL [npoints][nmaps], chi2, logdet [npoints], choice)."""
    pk = packed or pack_problem(p, device)
    if device:
        import torch
        clp = cl_points if _is_torch(cl_points) else torch.as_tensor(np.ascontiguousarray(cl_points, np.float64))
        clp = clp.to("cuda", torch.float64).contiguous()
        m = maps if _is_torch(maps) else torch.as_tensor(np.ascontiguousarray(maps, np.float64))
        m = torch.atleast_2d(m.to("cuda", torch.float64)).contiguous()
    else:
        clp = _host(cl_points)
        m = np.atleast_2d(_host(maps))
    npoints, lstride, nmaps = int(clp.shape[0]), int(clp.shape[-1]), int(m.shape[0])
    m2 = _alloc((npoints, nmaps), device)
    x2 = _alloc((npoints, nmaps), device)
    ld = _alloc((npoints,), device)
    ch = cf_basis_choice()
    rep = cf_report()
    ex = _exec(_torch_stream() if device else None)
    st = lib().cf_loglike_auto(C.byref(pk.struct), int(window[0]), int(window[1]), _field_bits(fields), npoints,
                               _ptr(clp), lstride, _ptr(m), nmaps, _ptr(m2), _ptr(x2), _ptr(ld), C.byref(ch),
                               C.byref(ex), C.byref(rep))
    _check(st, rep)
    out = {"m2lnL": m2, "chi2": x2, "logdet": ld, "choice": ch.as_dict()}
    return (out, rep.as_dict()) if report else out


# ------------------------------------------------------------------------------ emulator
def qml_iterate(p, bins, data, max_iter=20, tol=1e-6, device=False, report=False, packed=None):
    """Iterative QML of one map [n]: dict(chat [K], F [K][K] at the last fiducial, cl [6][lmax+1]
    (host) the last fiducial, iterations)."""
    pk = packed or pack_problem(p, device)
    bs, keep = pack_bins(bins)
    K = len(bins.spectra) * bs.nbins
    if device:
        import torch
        d = data if _is_torch(data) else torch.as_tensor(np.ascontiguousarray(data, np.float64))
        d = d.to("cuda", torch.float64).contiguous().reshape(-1)
    else:
        d = np.ascontiguousarray(_host(data).reshape(-1))
    chat, F = _alloc((K,), device), _alloc((K, K), device)
    cl = np.zeros((6, p.lmax + 1))
    iters = C.c_int32(0)
    rep = cf_report()
    ex = _exec(_torch_stream() if device else None)
    st = lib().cf_qml_iterate(C.byref(pk.struct), C.byref(bs), _ptr(d), int(max_iter), C.c_double(tol),
                              _ptr(chat), _ptr(F), _ptr(cl), C.byref(iters), C.byref(ex), C.byref(rep))
    _check(st, rep)
    out = {"chat": chat, "F": F, "cl": cl, "iterations": int(iters.value)}
    return (out, rep.as_dict()) if report else out


def decorrelate(F, q=None, device=False, report=False):
    """Decorrelated estimates F^-1/2 q (Eq. decorrelated) for each row of q, and F^-1/2 itself.
    Returns (out [nvec][K] or None, Fmhalf [K][K])."""
    if device:
        import torch
        Fd = (F if _is_torch(F) else torch.as_tensor(np.ascontiguousarray(F, np.float64))).to("cuda", torch.float64).contiguous()
        qd = None if q is None else torch.atleast_2d((q if _is_torch(q) else torch.as_tensor(np.ascontiguousarray(q, np.float64))).to("cuda", torch.float64)).contiguous()
    else:
        Fd = _host(F)
        qd = None if q is None else np.atleast_2d(_host(q))
    K = int(Fd.shape[0])
    nvec = 0 if qd is None else int(qd.shape[0])
    out = _alloc((nvec, K), device) if nvec else None
    R = _alloc((K, K), device)
    rep = cf_report()
    ex = _exec(_torch_stream() if device else None)
    st = lib().cf_decorrelate(_ptr(Fd), K, _ptr(qd), nvec, CF_MEM_DEVICE if device else CF_MEM_HOST,
                              _ptr(out), _ptr(R), C.byref(ex), C.byref(rep))
    _check(st, rep)
    return ((out, R), rep.as_dict()) if report else (out, R)


FIELD_BITS = {"T": 1, "E": 2, "B": 4}


class SMW:
    """Pixel likelihood through the harmonic basis with multipole switching (cf_smw_*).

    The window is the multipole range ``window = (lo, hi)`` on the harmonic fields ``fields``
    (default: all of the problem's).  Construction factors N_eff and solves the maps and the
    window's harmonic rows against it; ``loglike`` then evaluates -2 ln L at points whose spectra
    differ from the problem's only inside the window, at the cost of a factorisation of the
    window's size per point."""

    def __init__(self, problem, maps, window, fields=None, device=False, packed=None):
        pk = packed or pack_problem(problem, device)
        if fields is None:
            fields = {"T": "T", "QU": "EB", "TQU": "TEB"}[problem.fields]
        bits = sum(FIELD_BITS[f] for f in set(fields))
        if device:
            import torch
            m = maps if _is_torch(maps) else torch.as_tensor(np.ascontiguousarray(maps, np.float64))
            m = torch.atleast_2d(m.to("cuda", torch.float64)).contiguous()
        else:
            m = np.atleast_2d(_host(maps))
        self.device = device
        self.nmaps = int(m.shape[0])
        self.lmax = int(problem.lmax)
        h = C.c_void_p()
        rep = cf_report()
        ex = _exec(_torch_stream() if device else None)
        st = lib().cf_smw_create(C.byref(pk.struct), int(window[0]), int(window[1]), bits, _ptr(m),
                                 self.nmaps, C.byref(ex), C.byref(h), C.byref(rep))
        _check(st, rep)
        self._h = h
        self.setup_report = rep.as_dict()

    @property
    def dim(self) -> int:
        return int(lib().cf_smw_dim(self._h))

    def loglike(self, cl_points, stage_timing=False, report=False):
        """-2 ln L [npoints][nmaps], chi^2 (same) and ln|C| [npoints]; cl_points [npoints][6][lstride]."""
        if not self._h:
            raise CFError(CF_EINVAL, "handle closed", None)
        if self.device:
            import torch
            clp = cl_points if _is_torch(cl_points) else torch.as_tensor(np.ascontiguousarray(cl_points, np.float64))
            clp = clp.to("cuda", torch.float64).contiguous()
        else:
            clp = _host(cl_points)
        npoints, lstride = int(clp.shape[0]), int(clp.shape[-1])
        assert clp.shape[1] == 6
        m2 = _alloc((npoints, self.nmaps), self.device)
        x2 = _alloc((npoints, self.nmaps), self.device)
        ld = _alloc((npoints,), self.device)
        rep = cf_report()
        ex = _exec(_torch_stream() if self.device else None, stage_timing)
        st = lib().cf_smw_loglike(self._h, npoints, _ptr(clp), lstride, _ptr(m2), _ptr(x2), _ptr(ld),
                                  C.byref(ex), C.byref(rep))
        _check(st, rep)
        out = {"m2lnL": m2, "chi2": x2, "logdet": ld}
        return (out, rep.as_dict()) if report else out

    def close(self):
        if getattr(self, "_h", None):
            lib().cf_smw_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Emulator:
    """Handle of a cf_emu ensemble (see include/cf.h); every method is one library call."""

    def __init__(self, in_dim=7, width=256, depth=3, ensemble=4, seed=501, _handle=None):
        self._h = C.c_void_p()
        if _handle is not None:
            self._h = _handle
        else:
            _check(lib().cf_emu_create(in_dim, width, depth, ensemble, seed, C.byref(self._h)))
        v = [C.c_int32() for _ in range(4)]
        _check(lib().cf_emu_shape(self._h, *[C.byref(a) for a in v]))
        self.in_dim, self.width, self.depth, self.ensemble = (a.value for a in v)
        self.P = int(lib().cf_emu_param_count(self._h))

    @classmethod
    def load(cls, path):
        h = C.c_void_p()
        _check(lib().cf_emu_load(str(path).encode(), C.byref(h)))
        return cls(_handle=h)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.cf_emu_destroy(h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def save(self, path):
        _check(lib().cf_emu_save(self._h, str(path).encode()))

    def train(self, x, y, epochs=200, batch=1024, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              val_frac=0.1, baseline=2, device=False, report=False):
        xs, ys = self._arr(x, device), self._arr(y, device)
        o = cf_emu_opts(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps),
                        float(val_frac), int(baseline))
        rep = cf_report()
        ex = _exec(_torch_stream() if device else None)
        st = lib().cf_emu_train(self._h, _ptr(xs), _ptr(ys), xs.shape[0],
                                CF_MEM_DEVICE if device else CF_MEM_HOST, C.byref(o), C.byref(ex),
                                C.byref(rep))
        _check(st, rep)
        return rep.as_dict() if report else None

    def predict(self, x, spread_max=0.1, exact=None, device=False, report=False, exact_smw=None):
        """exact = (problem, base [6][L], basis [in][6][L], map [n]) enables the exact fallback
        through the pixel likelihood; exact_smw = (SMW handle with one map, base, basis) through the
        harmonic-basis likelihood.  Returns dict(y, spread, fallback)."""
        xs = self._arr(x, device)
        N = xs.shape[0]
        keep = []
        pp = ms = mp = None
        if exact_smw is not None:
            h, base, basis = exact_smw
            base, basis = _host(base), _host(basis)
            keep += [base, basis]
            ms = C.byref(cf_linear_spectra(basis.shape[0], base.shape[-1], _ptr(base), _ptr(basis)))
        elif exact is not None:
            prob, base, basis, emap = exact
            pk = pack_problem(prob, device)
            keep.append(pk)
            pp = C.byref(pk.struct)
            base, basis = _host(base), _host(basis)
            keep += [base, basis]
            ms = cf_linear_spectra(basis.shape[0], base.shape[-1], _ptr(base), _ptr(basis))
            ms = C.byref(ms)
            em = self._arr(emap, device)
            keep.append(em)
            mp = _ptr(em)
        y = _alloc((N,), device)
        sp = _alloc((N,), device)
        if device:
            import torch
            fb = torch.empty((N,), dtype=torch.uint8, device="cuda")
        else:
            fb = np.empty((N,), dtype=np.uint8)
        rep = cf_report()
        ex = _exec(_torch_stream() if device else None)
        if exact_smw is not None:
            st = lib().cf_emu_predict_smw(self._h, _ptr(xs), N, CF_MEM_DEVICE if device else CF_MEM_HOST,
                                          float(spread_max), exact_smw[0]._h, ms, _ptr(y), _ptr(sp),
                                          _ptr(fb, C.c_uint8), C.byref(ex), C.byref(rep))
        else:
            st = lib().cf_emu_predict(self._h, _ptr(xs), N, CF_MEM_DEVICE if device else CF_MEM_HOST,
                                      float(spread_max), pp, ms, mp, _ptr(y), _ptr(sp),
                                      _ptr(fb, C.c_uint8), C.byref(ex), C.byref(rep))
        _check(st, rep)
        out = {"y": y, "spread": sp, "fallback": fb}
        return (out, rep.as_dict()) if report else out

    def get_params(self, member=0):
        out = np.empty(self.P, np.float32)
        _check(lib().cf_emu_get_params(self._h, member, _ptr(out, C.c_float)))
        return out

    def set_params(self, member, p):
        p = _host(p, np.float32)
        assert p.shape == (self.P,)
        _check(lib().cf_emu_set_params(self._h, member, _ptr(p, C.c_float)))

    def forward(self, xn):
        xn = _host(xn)
        N = xn.shape[0]
        out = np.empty((self.ensemble, N), np.float32)
        _check(lib().cf_emu_forward(self._h, _ptr(xn), N, _ptr(out, C.c_float)))
        return out

    def gradient(self, xn, yn):
        xn, yn = _host(xn), _host(yn)
        N = xn.shape[0]
        g = np.empty((self.ensemble, self.P), np.float32)
        loss = np.empty(self.ensemble, np.float64)
        _check(lib().cf_emu_gradient(self._h, _ptr(xn), _ptr(yn), N, _ptr(g, C.c_float), _ptr(loss)))
        return g, loss

    def adam(self, grad, lr):
        g = _host(grad, np.float32)
        _check(lib().cf_emu_adam(self._h, _ptr(g, C.c_float), float(lr)))

    @staticmethod
    def _arr(a, device):
        if device:
            import torch
            t = a if _is_torch(a) else torch.as_tensor(np.ascontiguousarray(a, np.float64))
            return t.to("cuda", torch.float64).contiguous()
        return _host(a)
