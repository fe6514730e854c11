"""CPU-side checks of the C ABI: the library loads, exports every function that
include/msbfm.h declares, and its host-only entry points behave (no GPU needed)."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2301_11828_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    import paper_2301_11828_amd as msb
    return msb.load_library()


def _declared():
    src = open(os.path.join(ROOT, "include", "msbfm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(msb_[a-z_]+)\s*\(", src)))


def test_header_declares_the_api():
    names = _declared()
    for n in ("msb_plan_create", "msb_apply", "msb_solve_static", "msb_vv_run", "msb_grad_infl"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2301_11828_amd import build as B
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    import paper_2301_11828_amd as msb
    assert set(msb.EXPORTS) == set(_declared())


def test_crack_to_bonds_matches_oracle(lib):
    """Host entry point vs the oracle's independent brute force, bit-exact sets."""
    import oracle as O
    import paper_2301_11828_amd as msb
    from paper_2301_11828_amd import workloads as W
    for n, M, seg in [((40, 30), 3, [[0.21, 0.13, 0.77, 0.61]]),
                      ((64, 64), 4, W.crack_segment((0.5, 0.5), 0.3, 30.0)),
                      ((25, 25), 2, [[0.1, 0.5, 0.9, 0.5], [0.5, 0.1, 0.5, 0.9]])]:
        h = 1.0 / max(n)
        a = msb.crack_to_bonds(n, h, M, seg)
        b = O.crack_to_bonds(O.Problem(n, h, M, 1.0), seg)
        assert len(a) > 0 and np.array_equal(a, b)


def test_host_validation_errors(lib):
    """Invalid descriptions are rejected with MSB_EINVAL before any device work."""
    import ctypes
    import paper_2301_11828_amd as msb
    d, keep = msb._desc((10, 10), 0.1, 0, 1.0, (), 1.0, 1)      # M = 0 invalid
    nb = ctypes.c_int64(0)
    st = lib.msb_crack_to_bonds(ctypes.byref(d), None, 0, None, 0, ctypes.byref(nb))
    assert st == msb.MSB_EINVAL
    assert b"M must be" in lib.msb_last_error()
    d, keep = msb._desc((10, 10, 10), 0.1, 2, 1.0, (), 1.0, 1)
    st = lib.msb_crack_to_bonds(ctypes.byref(d), None, 0, None, 0, ctypes.byref(nb))
    assert st == msb.MSB_EUNSUPPORTED                           # cracks are 2D only
    p = ctypes.c_void_p()
    st = lib.msb_plan_create(None, ctypes.byref(p))
    assert st == msb.MSB_EINVAL and not p


def test_capacity_error_reports_count(lib):
    import ctypes
    import paper_2301_11828_amd as msb
    d, keep = msb._desc((30, 30), 1 / 30, 3, 1.0, (), 1.0, 1)
    seg = np.array([[0.2, 0.2, 0.8, 0.7]])
    nb = ctypes.c_int64(0)
    out = np.zeros((2, 2), dtype=np.int64)
    st = lib.msb_crack_to_bonds(ctypes.byref(d), seg.ctypes.data, 1, out.ctypes.data, 2, ctypes.byref(nb))
    assert st == msb.MSB_EINVAL and nb.value > 2


def test_workloads_have_no_method_arithmetic():
    """The shared input module is plain data generation (seeded); same seed, same data."""
    from paper_2301_11828_amd import workloads as W
    a, b = W.plate32(), W.plate32()
    assert np.array_equal(a.b, b.b) and np.array_equal(a.fixed, b.fixed)
    assert a.fixed.sum() == 2 * 348
