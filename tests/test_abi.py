"""C-ABI contract checks that need no GPU: the library loads, exports every symbol the header
declares, and rejects bad arguments before touching a device."""
import os
import re

import numpy as np
import pytest

from paper_2605_21149_amd import cf
from paper_2605_21149_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "cf.h")).read()
    return sorted(set(re.findall(r"^(?:const char\*|int64_t|int|void)\s+(cf_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    L = cf.lib()
    syms = _header_symbols()
    assert set(syms) == set(cf.EXPORTS)
    for name in syms:
        assert hasattr(L, name), name


def test_problem_dimensions():
    assert cf.problem_dim(I.spin0_problem_nside8()) == 544
    p = I.tqu_problem_nside16(dense_noise=False)
    assert cf.problem_dim(p) == 5952
    assert cf.problem_nmodes(p) == 3 * (48 * 48 - 4)
    assert cf.problem_dim(I.qu_problem_nside32()) == 12288


def _expect(code, fn):
    with pytest.raises(cf.CFError) as e:
        fn()
    assert e.value.status == code, str(e.value)
    return str(e.value)


def test_argument_validation():
    p = I.spin0_problem_nside8()
    bins = I.uniform_bins(2, 24, 1, ("TT",))
    # bin outside [lmin, lmax]
    bad = I.Bins(np.array([2]), np.array([25]), ("TT",))
    assert "outside" in _expect(cf.CF_EINVAL, lambda: cf.fisher(p, bad))
    # spectrum for an absent field
    assert "absent" in _expect(cf.CF_EINVAL, lambda: cf.fisher(p, I.Bins(bins.lo, bins.hi, ("EE",))))
    # NaN in the spectra
    q = I.spin0_problem_nside8()
    q.cl = q.cl.copy()
    q.cl[0, 5] = np.nan
    assert "non-finite" in _expect(cf.CF_EINVAL, lambda: cf.fisher(q, bins))
    # l-range chain: lmin < 2 with Q,U present
    r = I.qu_scan_problem(8)
    r.lmin = 1
    assert "spin" in _expect(cf.CF_EINVAL, lambda: cf.cov_build(r))
    # lmax < lmin
    r = I.spin0_problem_nside8()
    r.lmin, r.lmax = 5, 4
    _expect(cf.CF_EINVAL, lambda: cf.cov_build(r))
    # non-finite noise
    r = I.spin0_problem_nside8()
    r.noise_diag = r.noise_diag.copy()
    r.noise_diag[3] = np.inf
    assert "noise" in _expect(cf.CF_EINVAL, lambda: cf.cov_build(r))
    # an unknown precision is rejected, not silently run in FP64
    _expect(cf.CF_EINVAL, lambda: cf.fisher(p, bins, precision=7))


def test_emulator_argument_validation():
    """Shape checks of cf_emu_create run before any device call."""
    import ctypes as C
    L = cf.lib()
    h = C.c_void_p()
    for args in ((0, 256, 3, 4), (9, 256, 3, 4), (7, 96, 3, 4), (7, 256, 0, 4), (7, 256, 9, 4),
                 (7, 256, 3, 0), (7, 256, 3, 17)):
        assert L.cf_emu_create(*args, 1, C.byref(h)) == cf.CF_EINVAL
        assert not h.value
    assert L.cf_emu_param_count(None) == -1
    assert L.cf_emu_shape(None, None, None, None, None) == cf.CF_EINVAL
    assert L.cf_emu_train(None, None, None, 0, 0, None, None, None) == cf.CF_EINVAL
    assert L.cf_emu_load(b"/nonexistent/emu.bin", C.byref(h)) == cf.CF_EINVAL
    L.cf_emu_destroy(None)
