"""msb_grad_infl_noalloc: the gradient entry point that allocates no device memory (its
partials and per-case sums live in the library's fixed device array) against the
allocating msb_grad_infl, on two calls in a row, the second on a smaller plan."""
import ctypes

import numpy as np
import pytest

from paper_2301_11828_amd import workloads as W
from helpers import gpu_plan, log, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _raw_noalloc(plan, u, w):
    """Direct C-ABI call of msb_grad_infl_noalloc (status, dL/da)."""
    import torch
    import paper_2301_11828_amd as msb
    lib = msb.load_library()
    out = np.zeros((plan.batch, plan.n_infl), dtype=np.float64)
    st = lib.msb_grad_infl_noalloc(plan._ptr, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                   out.ctypes.data, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, out


def _case(n, M, batch, K, seed, tile=None):
    rng = np.random.default_rng(seed)
    a = tuple(rng.uniform(0.2, 1.0, size=K))
    w = W.small(2, n, M, seed=seed, fixed="all", crack=True, batch=batch, infl=a)
    plan = gpu_plan(w)
    if tile:
        plan.set_config("fp64", **tile)
    u = to_dev(w.b)
    wv = to_dev(rng.standard_normal((batch, 2, w.N)))
    return plan, u, wv


@pytest.mark.parametrize("tile", [None, dict(tile=16, tile_regs=1), dict(tile=24, tile_regs=0)])
def test_noalloc_gradient_equals_allocating_gradient_twice(tile):
    import paper_2301_11828_amd as msb
    big = _case((64, 57), 3, 2, 6, 801, tile)
    small = _case((33, 29), 2, 1, 3, 802, tile)
    refs = [p.grad_infl(u, wv) for p, u, wv in (big, small)]     # builds the derivative operators
    for (p, u, wv), ref in zip((big, small), refs):
        st, g = _raw_noalloc(p, u, wv)
        assert st == msb.MSB_OK, msb.load_library().msb_last_error()
        err = rel_err(g, ref)
        log("noalloc gradient %s batch %d: rel diff vs msb_grad_infl %.2e" % (p.n, p.batch, err))
        assert g.shape == ref.shape and err <= 1e-12
    # and once more on the larger plan after the smaller one left its values in the array
    st, g = _raw_noalloc(*big)
    assert st == msb.MSB_OK and rel_err(g, refs[0]) <= 1e-12


def test_noalloc_gradient_rejections():
    import paper_2301_11828_amd as msb
    # derivative operators not built yet
    p, u, wv = _case((30, 27), 3, 1, 2, 803)
    st, _ = _raw_noalloc(p, u, wv)
    assert st == msb.MSB_EINVAL
    assert "derivative operator" in msb.load_library().msb_last_error().decode()
    # more partials than the fixed array holds: 1800 cases x 200 row partials x 3 > 2^20
    B = 1800
    w = W.small(2, (50, 200), 1, seed=804, batch=1, infl=(0.5,))
    plan = msb.Plan(w.n, w.h, w.M, w.alpha, infl=w.infl, batch=B)
    plan.set_config("fp64", rows_per_wg=1, team_x=0)
    import torch
    u = torch.zeros((B, 2, w.N), dtype=torch.float64, device="cuda")
    plan.apply_dinfl(0, u)
    st, _ = _raw_noalloc(plan, u, u)
    assert st == msb.MSB_EINVAL
    msg = msb.load_library().msb_last_error().decode()
    log("oversize rejection: %s" % msg)
    assert "scratch" in msg
