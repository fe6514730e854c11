"""MI355X (gfx950) implementation of the matrix-structure-based fast method (MSBFM)
for linear bond-based peridynamics (Liu, Tian, Don, Wang, arXiv 2301.11828).

This module is a thin ctypes binding over ``libmsbfm.so`` (C ABI in
``include/msbfm.h``): it checks and marshals arguments, and PyTorch supplies device
memory and the current stream.  Every step of the computation runs in the library's
HIP kernels; there is no CPU fallback, and importing fails loudly when the library
has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libmsbfm.so")

MSB_OK, MSB_EINVAL, MSB_ENOMEM, MSB_EDEVICE, MSB_ENOCONV, MSB_ENOTSPD, MSB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FP64, FP32, FP32_REFINED = 0, 1, 2
_STATUS = {0: "MSB_OK", -1: "MSB_EINVAL", -2: "MSB_ENOMEM", -3: "MSB_EDEVICE", -4: "MSB_ENOCONV",
           -5: "MSB_ENOTSPD", -6: "MSB_EUNSUPPORTED"}

# every symbol include/msbfm.h declares
EXPORTS = ("msb_plan_create", "msb_plan_destroy", "msb_plan_set_constraints", "msb_plan_set_bonds",
           "msb_crack_to_bonds", "msb_plan_set_infl", "msb_apply", "msb_apply_dinfl", "msb_apply_precond",
           "msb_crack_update", "msb_plan_get_bonds", "msb_plan_set_surface", "msb_surface_volume_factors",
           "msb_adr_run",
           "msb_solve_static", "msb_vv_init", "msb_vv_run", "msb_grad_infl", "msb_grad_infl_noalloc",
           "msb_plan_info",
           "msb_profile_apply", "msb_plan_get_config", "msb_plan_set_config", "msb_plan_set_lengths",
           "msb_plan_autotune", "msb_group_create", "msb_group_destroy", "msb_group_get_config",
           "msb_group_set_config", "msb_group_apply", "msb_group_set_infl", "msb_group_autotune",
           "msb_group_solve_static",
           "msb_last_error")


class MsbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double),
                ("M", ctypes.c_int), ("alpha", ctypes.c_double), ("n_infl", ctypes.c_int),
                ("infl", ctypes.POINTER(ctypes.c_double)), ("rho", ctypes.c_double),
                ("batch", ctypes.c_int)]


class _Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("graph_block", ctypes.c_int), ("reliable_update", ctypes.c_int), ("precond", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("outer_iters", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


class _LaunchConfig(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int) for k in ("rows_per_wg", "team_x", "slots_fwd", "slots_inv", "threads_x",
                                            "lines_per_wg", "team_line", "lines_per_wave", "threads_line",
                                            "max_radix", "lds_inplace", "tile", "threads_tile", "tile_regs",
                                            "tile_run")]


CONFIG_KEYS = tuple(k for k, _ in _LaunchConfig._fields_)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmsbfm.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libmsbfm.so not built (expected at %s); run python -m paper_2301_11828_amd.build"
                          % path)
    # One HIP runtime per process: let PyTorch load (and initialise) its runtime first so
    # that the library's libamdhip64.so.7 dependency binds to that same copy.
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "msb_plan_create": ([ctypes.POINTER(_Desc), ctypes.POINTER(P)], I),
        "msb_plan_destroy": ([P], None),
        "msb_plan_set_constraints": ([P, P], I),
        "msb_plan_set_bonds": ([P, P, I64], I),
        "msb_crack_to_bonds": ([ctypes.POINTER(_Desc), P, I64, P, I64, ctypes.POINTER(I64)], I),
        "msb_plan_set_infl": ([P, P, I, I], I),
        "msb_apply": ([P, I, P, P, P], I),
        "msb_apply_dinfl": ([P, I, P, P, P], I),
        "msb_apply_precond": ([P, I, P, P, P], I),
        "msb_crack_update": ([P, I, P, D, ctypes.POINTER(I64), P], I),
        "msb_plan_get_bonds": ([P, P, I64, ctypes.POINTER(I64)], I),
        "msb_plan_set_surface": ([P, P], I),
        "msb_adr_run": ([P, I, I64, I, P, P, P, P, P, P, P], I),
        "msb_surface_volume_factors": ([P, P], I),
        "msb_solve_static": ([P, I, P, P, P, ctypes.POINTER(_Opts), P, P], I),
        "msb_vv_init": ([P, I, P, P, P, P], I),
        "msb_vv_run": ([P, I, D, I64, P, P, P, P, P, P, I, P], I),
        "msb_grad_infl": ([P, P, P, P, P], I),
        "msb_grad_infl_noalloc": ([P, P, P, P, P], I),
        "msb_plan_info": ([P, P, P, P], I),
        "msb_profile_apply": ([P, I, P, P, I, P, P, P], I),
        "msb_plan_get_config": ([P, I, ctypes.POINTER(_LaunchConfig)], I),
        "msb_plan_set_config": ([P, I, ctypes.POINTER(_LaunchConfig)], I),
        "msb_plan_set_lengths": ([P, P], I),
        "msb_plan_autotune": ([P, I, I, I, ctypes.POINTER(_LaunchConfig), ctypes.POINTER(D), P], I),
        "msb_group_create": ([P, I, ctypes.POINTER(P)], I),
        "msb_group_destroy": ([P], None),
        "msb_group_get_config": ([P, I, ctypes.POINTER(_LaunchConfig)], I),
        "msb_group_set_config": ([P, I, ctypes.POINTER(_LaunchConfig)], I),
        "msb_group_apply": ([P, I, P, P, P], I),
        "msb_group_set_infl": ([P, P, I, P], I),
        "msb_group_autotune": ([P, I, I, ctypes.POINTER(_LaunchConfig), ctypes.POINTER(D)], I),
        "msb_group_solve_static": ([P, I, P, P, P, ctypes.POINTER(_Opts), P, P], I),
        "msb_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(st: int):
    if st != MSB_OK:
        raise MsbError(st, _lib.msb_last_error().decode())


def _desc(n: Sequence[int], h: float, M: int, alpha: float, infl, rho: float, batch: int):
    d = _Desc()
    d.dim = len(n)
    if d.dim not in (2, 3):
        raise ValueError("grid must be 2D or 3D")
    for a in range(3):
        d.n[a] = int(n[a]) if a < len(n) else 1
    d.h, d.M, d.alpha, d.rho, d.batch = float(h), int(M), float(alpha), float(rho), int(batch)
    arr = np.ascontiguousarray(np.asarray(infl, dtype=np.float64))
    d.n_infl = len(arr)
    d.infl = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if len(arr) else None
    return d, arr


def crack_to_bonds(n: Sequence[int], h: float, M: int, segments) -> np.ndarray:
    """Broken bonds of 2D crack segments [(x0, y0, x1, y1), ...] (host computation)."""
    lib = load_library()
    d, _keep = _desc(n, h, M, 1.0, (), 1.0, 1)
    seg = np.ascontiguousarray(np.asarray(segments, dtype=np.float64).reshape(-1, 4))
    nb = ctypes.c_int64(0)
    st = lib.msb_crack_to_bonds(ctypes.byref(d), seg.ctypes.data, len(seg), None, 0, ctypes.byref(nb))
    if st not in (MSB_OK, MSB_EINVAL) or (st == MSB_EINVAL and nb.value == 0):
        _check(st)
    out = np.zeros((max(nb.value, 1), 2), dtype=np.int64)
    _check(lib.msb_crack_to_bonds(ctypes.byref(d), seg.ctypes.data, len(seg), out.ctypes.data,
                                  nb.value, ctypes.byref(nb)))
    return out[:nb.value]


@dataclass
class SolveInfo:
    status: int
    outer_iters: int
    inner_iters: int
    rel_residual: float
    seconds: float


def _torch():
    import torch
    return torch


def loaded_hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process (diagnostics)."""
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                paths.add(line.split()[-1])
    return sorted(paths)


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_PREC = {"fp64": FP64, "fp32": FP32, "fp32_refined": FP32_REFINED}


class Plan:
    """A grid, horizon and operator (A = A_hat + D^e + D^f, masked rows) on the current GPU.

    n      -- (nx, ny) or (nx, ny, nz) nodes; node (i,j,k) at ((i+1/2)h, ...)
    h, M   -- spacing and horizon in cells (delta = M h)
    alpha  -- micromodulus scale (9E/(pi delta^3) in 2D, 12E/(pi delta^4) in 3D)
    infl   -- optional coefficients a_k of omega(r) = sum_k a_k (r/delta)^k
    batch  -- number of load cases sharing the plan; vectors are [batch, dim, N]
    """

    def __init__(self, n: Sequence[int], h: float, M: int, alpha: float, infl=(), rho: float = 1.0,
                 batch: int = 1):
        lib = load_library()
        self.n = tuple(int(x) for x in n)
        self.dim = len(self.n)
        self.N = int(np.prod(self.n))
        self.batch = int(batch)
        self.M = int(M)
        self.h = float(h)
        self.n_infl = len(infl)
        d, keep = _desc(self.n, h, M, alpha, infl, rho, batch)
        self._ptr = ctypes.c_void_p()
        _check(lib.msb_plan_create(ctypes.byref(d), ctypes.byref(self._ptr)))
        del keep
        # what the operator was last built from, so that an adjoint solve can check it
        # still applies the operator of its forward solve: the coefficients (restored
        # when they differ) and a count of the other operator changes (constraints,
        # broken bonds, surface factors), which it cannot restore
        self._infl_state = (np.array(infl, dtype=np.float64), False)
        self._struct_version = 0
        self.graph_block = 0   # default of solve(): CG iterations per hipGraph launch (0: none)

    def close(self):
        if self._ptr:
            _lib.msb_plan_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ configuration
    @property
    def padded_lengths(self):
        L = (ctypes.c_int64 * 3)()
        _check(_lib.msb_plan_info(self._ptr, L, None, None))
        return tuple(L[:self.dim])

    @property
    def n_bonds(self) -> int:
        nb = ctypes.c_int64()
        _check(_lib.msb_plan_info(self._ptr, None, None, ctypes.byref(nb)))
        return nb.value

    def get_config(self, precision: str = "fp64") -> dict:
        """Launch configuration of the product kernels for "fp64" or "fp32" (a dict
        with the fields of msb_launch_config)."""
        c = _LaunchConfig()
        _check(_lib.msb_plan_get_config(self._ptr, _PREC[precision], ctypes.byref(c)))
        return {k: getattr(c, k) for k in CONFIG_KEYS}

    def set_config(self, precision: str = "fp64", **fields):
        """Change some fields of the launch configuration (validated by the library)."""
        c = _LaunchConfig()
        _check(_lib.msb_plan_get_config(self._ptr, _PREC[precision], ctypes.byref(c)))
        for k, v in fields.items():
            if k not in CONFIG_KEYS:
                raise KeyError("unknown launch configuration field %r" % k)
            setattr(c, k, int(v))
        _check(_lib.msb_plan_set_config(self._ptr, _PREC[precision], ctypes.byref(c)))

    def set_lengths(self, L: Sequence[int]):
        """New zero-padded transform lengths (each >= N + M, factors 2, 3, 5 only)."""
        arr = (ctypes.c_int64 * 3)(*([int(x) for x in L] + [1] * (3 - len(L))))
        _check(_lib.msb_plan_set_lengths(self._ptr, arr))

    def autotune(self, precision: str = "fp64", effort: int = 1, lengths: bool = False):
        """Time candidate launch configurations (and, with lengths=True, padded
        lengths) and keep the fastest.  Returns (configuration dict, product ms)."""
        c = _LaunchConfig()
        ms = ctypes.c_double(0.0)
        _check(_lib.msb_plan_autotune(self._ptr, _PREC[precision], int(effort), int(bool(lengths)),
                                      ctypes.byref(c), ctypes.byref(ms), _stream()))
        return {k: getattr(c, k) for k in CONFIG_KEYS}, ms.value

    def set_constraints(self, fixed: Optional[np.ndarray]):
        if fixed is None:
            _check(_lib.msb_plan_set_constraints(self._ptr, None))
            self._struct_version += 1
            return
        f = np.ascontiguousarray(np.asarray(fixed).reshape(self.dim, self.N).astype(np.uint8))
        _check(_lib.msb_plan_set_constraints(self._ptr, f.ctypes.data))
        self._struct_version += 1

    def set_bonds(self, pairs: Optional[np.ndarray]):
        p = np.ascontiguousarray(np.asarray(pairs if pairs is not None else np.zeros((0, 2)),
                                            dtype=np.int64).reshape(-1, 2))
        _check(_lib.msb_plan_set_bonds(self._ptr, p.ctypes.data if len(p) else None, len(p)))
        self._struct_version += 1

    def set_surface(self, nu: Optional[np.ndarray]):
        """Surface-correction factors per node ([N], or None to switch the correction off)."""
        self._struct_version += 1
        if nu is None:
            _check(_lib.msb_plan_set_surface(self._ptr, None))
            return
        a = np.ascontiguousarray(np.asarray(nu, dtype=np.float64).reshape(-1))
        if a.size != self.N:
            raise ValueError("nu must hold N = %d values" % self.N)
        _check(_lib.msb_plan_set_surface(self._ptr, a.ctypes.data))

    def surface_volume_factors(self) -> np.ndarray:
        out = np.empty(self.N, dtype=np.float64)
        _check(_lib.msb_surface_volume_factors(self._ptr, out.ctypes.data))
        return out

    def bonds(self) -> np.ndarray:
        """The broken set as [n][2] int64 pairs (p < q), sorted."""
        cnt = ctypes.c_int64()
        _check(_lib.msb_plan_get_bonds(self._ptr, None, 0, ctypes.byref(cnt)))
        out = np.zeros((cnt.value, 2), dtype=np.int64)
        if cnt.value:
            _check(_lib.msb_plan_get_bonds(self._ptr, out.ctypes.data, cnt.value, ctypes.byref(cnt)))
        return out

    def crack_update(self, u, s0: float) -> int:
        """Break every bond whose stretch (eq. (fra:s1)) reaches s0; returns the number of new breaks."""
        torch = _torch()
        prec = FP64 if u.dtype == torch.float64 else FP32
        n = ctypes.c_int64()
        _check(_lib.msb_crack_update(self._ptr, prec, self._vec(u, u.dtype, "u"), float(s0), ctypes.byref(n),
                                     _stream()))
        if n.value:
            self._struct_version += 1
        return n.value

    def set_infl(self, infl, per_case: bool = False):
        a = np.ascontiguousarray(np.asarray(infl, dtype=np.float64))
        k = a.shape[-1] if a.ndim else 0
        _check(_lib.msb_plan_set_infl(self._ptr, a.ctypes.data, int(k), int(per_case)))
        self.n_infl = int(k)
        self._infl_state = (a.copy(), bool(per_case))

    def _operator_state(self):
        return (self._infl_state[0].copy(), self._infl_state[1], self._struct_version)

    def _restore_operator(self, state):
        """Make the plan apply the operator recorded by _operator_state() again: the
        coefficients are re-applied when they differ; any other operator change since
        then cannot be undone and raises.  Returns the state to restore afterwards, or
        None when nothing changed."""
        infl, per_case, version = state
        if version != self._struct_version:
            raise RuntimeError("the plan's constraints, broken bonds or surface factors changed between the "
                               "forward solve and its adjoint")
        cur = self._infl_state
        if cur[1] == per_case and cur[0].shape == infl.shape and np.array_equal(cur[0], infl):
            return None
        before = self._operator_state()
        self.set_infl(infl, per_case=per_case)
        return before

    # ------------------------------------------------------------ tensors
    def _vec(self, t, dtype=None, name="vector"):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA (HIP) tensor" % name)
        if dtype is not None and t.dtype != dtype:
            raise TypeError("%s must be %s" % (name, dtype))
        if t.numel() != self.batch * self.dim * self.N:
            raise ValueError("%s must hold batch*dim*N = %d values" % (name, self.batch * self.dim * self.N))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        return ctypes.c_void_p(t.data_ptr())

    def empty(self, dtype=None):
        torch = _torch()
        return torch.empty((self.batch, self.dim, self.N), dtype=dtype or torch.float64, device="cuda")

    # ------------------------------------------------------------ operations
    def apply(self, u, out=None):
        """f = A u on free DOFs, 0 on constrained ones (FP64 for float64, FP32 for float32)."""
        torch = _torch()
        prec = FP64 if u.dtype == torch.float64 else FP32
        if out is None:
            out = torch.empty_like(u)
        _check(_lib.msb_apply(self._ptr, prec, self._vec(u, u.dtype, "u"), self._vec(out, u.dtype, "out"),
                              _stream()))
        return out

    def apply_dinfl(self, k: int, u, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty_like(u)
        _check(_lib.msb_apply_dinfl(self._ptr, int(k), self._vec(u, torch.float64, "u"),
                                    self._vec(out, torch.float64, "out"), _stream()))
        return out

    def apply_precond(self, r, out=None):
        """z = C^{-1} r of the preconditioned solver (masked to free DOFs); fp64 or fp32 by r's dtype."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(r)
        prec = FP64 if r.dtype == torch.float64 else FP32
        _check(_lib.msb_apply_precond(self._ptr, prec, self._vec(r, r.dtype, "r"), self._vec(out, r.dtype, "out"),
                                      _stream()))
        return out

    def solve(self, b, g=None, precision: str = "fp64", tol: float = 1e-10, maxit: int = 100000,
              inner_tol: float = 0.0, graph_block=None, reliable_update: int = 0, out=None,
              check: bool = True, precond: bool = False):
        """Static model: K u = b on free DOFs, u = g on constrained (K = -A).  Returns (u, infos).
        precond: CG preconditioned by the circulant inverse of the periodic operator;
        graph_block: CG iterations per hipGraph launch (None: the plan's `graph_block`
        attribute, 0 unless set, which the autograd function's solves also use)."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(b)
        gb = self.graph_block if graph_block is None else int(graph_block)
        opts = _Opts(tol, int(maxit), float(inner_tol), gb, int(reliable_update), int(bool(precond)))
        infos = (_Info * self.batch)()
        gp = self._vec(g, torch.float64, "g") if g is not None else None
        st = _lib.msb_solve_static(self._ptr, _PREC[precision], self._vec(b, torch.float64, "b"), gp,
                                   self._vec(out, torch.float64, "u"), ctypes.byref(opts), infos, _stream())
        res = [SolveInfo(i.status, i.outer_iters, i.inner_iters, i.rel_residual, i.seconds) for i in infos]
        if check:
            _check(st)
        return out, res

    def adr_run(self, nsteps: int, u, v, F, b, g=None, restart: bool = True, residual: bool = False):
        """Adaptive dynamic relaxation (Alg. 1): nsteps updates of u (in place), velocity v and
        force F = A u + b; restart starts from u, else continues.  Returns ||F|| per case when
        residual is set."""
        torch = _torch()
        prec = FP64 if u.dtype == torch.float64 else FP32
        res = np.zeros(self.batch, dtype=np.float64) if residual else None
        gp = self._vec(g, u.dtype, "g") if g is not None else None
        _check(_lib.msb_adr_run(self._ptr, prec, int(nsteps), int(bool(restart)), self._vec(u, u.dtype, "u"),
                                self._vec(v, u.dtype, "v"), self._vec(F, u.dtype, "F"), self._vec(b, u.dtype, "b"),
                                gp, res.ctypes.data if res is not None else None, _stream()))
        return res

    def vv_init(self, u, b, a=None):
        torch = _torch()
        prec = FP64 if u.dtype == torch.float64 else FP32
        if a is None:
            a = torch.empty_like(u)
        _check(_lib.msb_vv_init(self._ptr, prec, self._vec(u, u.dtype, "u"), self._vec(b, u.dtype, "b"),
                                self._vec(a, u.dtype, "a"), _stream()))
        return a

    def vv_run(self, dt: float, nsteps: int, u, v, a, b, g=None, energy_every: int = 0):
        """Advance u, v, a in place by nsteps of velocity Verlet; returns energies (numpy)."""
        torch = _torch()
        prec = FP64 if u.dtype == torch.float64 else FP32
        ne = nsteps // energy_every if energy_every else 0
        en = np.zeros(max(ne, 1), dtype=np.float64)
        gp = self._vec(g, u.dtype, "g") if g is not None else None
        _check(_lib.msb_vv_run(self._ptr, prec, float(dt), int(nsteps), self._vec(u, u.dtype, "u"),
                               self._vec(v, u.dtype, "v"), self._vec(a, u.dtype, "a"),
                               self._vec(b, u.dtype, "b"), gp, en.ctypes.data if ne else None,
                               int(energy_every), _stream()))
        return en[:ne]

    def profile_apply(self, u, out=None, nrep: int = 20):
        """Mean per-kernel durations (ms) of the product chain, timed with HIP events."""
        torch = _torch()
        prec = FP64 if u.dtype == torch.float64 else FP32
        if out is None:
            out = torch.empty_like(u)
        ms = np.zeros(8, dtype=np.float64)
        npass = ctypes.c_int(0)
        _check(_lib.msb_profile_apply(self._ptr, prec, self._vec(u, u.dtype, "u"), self._vec(out, u.dtype, "out"),
                                      int(nrep), ms.ctypes.data, ctypes.byref(npass), _stream()))
        return ms[:npass.value]

    def grad_infl(self, u, w, noalloc: bool = False) -> np.ndarray:
        """dL/da_k = w . (A_k u)_F for every case: [batch, n_infl].  noalloc: the variant
        that allocates no device memory (msb_grad_infl_noalloc; its derivative operators
        must exist already)."""
        torch = _torch()
        out = np.zeros((self.batch, self.n_infl), dtype=np.float64)
        fn = _lib.msb_grad_infl_noalloc if noalloc else _lib.msb_grad_infl
        _check(fn(self._ptr, self._vec(u, torch.float64, "u"), self._vec(w, torch.float64, "w"), out.ctypes.data,
                  _stream()))
        return out


class PlanGroup:
    """Several plans of the same dimension run as one launch per pass (msb_group_*).

    The plans stay usable on their own; the group holds references and must be closed
    (or dropped) before them.  Vectors are passed as lists, one tensor per member, each
    shaped as for that member's Plan."""

    def __init__(self, plans, precond: bool = False):
        lib = load_library()
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._ptr.value for p in self.plans])
        self._ptr = ctypes.c_void_p()
        _check(lib.msb_group_create(arr, len(self.plans), ctypes.byref(self._ptr)))
        self.total_cases = sum(p.batch for p in self.plans)
        self.precond = bool(precond)   # default of solve(): circulant-preconditioned CG
        self.graph_block = 0           # default of solve(): CG iterations per hipGraph launch (0: none)
        self.reliable_update = 0       # default of solve(): FP32_REFINED keeps the search direction

    def close(self):
        if self._ptr:
            _lib.msb_group_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_config(self, precision: str = "fp64") -> dict:
        c = _LaunchConfig()
        _check(_lib.msb_group_get_config(self._ptr, _PREC[precision], ctypes.byref(c)))
        return {k: getattr(c, k) for k in CONFIG_KEYS}

    def set_config(self, precision: str = "fp64", **fields):
        c = _LaunchConfig()
        _check(_lib.msb_group_get_config(self._ptr, _PREC[precision], ctypes.byref(c)))
        for k, v in fields.items():
            if k not in CONFIG_KEYS:
                raise KeyError("unknown launch configuration field %r" % k)
            setattr(c, k, int(v))
        _check(_lib.msb_group_set_config(self._ptr, _PREC[precision], ctypes.byref(c)))

    def _ptrs(self, ts, dtype, name):
        if len(ts) != len(self.plans):
            raise ValueError("%s: one tensor per member (%d)" % (name, len(self.plans)))
        return (ctypes.c_void_p * len(ts))(*[p._vec(t, dtype, "%s[%d]" % (name, i)).value
                                             for i, (p, t) in enumerate(zip(self.plans, ts))])

    def apply(self, us, outs=None):
        """f_i = A_i u_i for every member (float64 -> FP64, float32 -> FP32)."""
        torch = _torch()
        dt = us[0].dtype
        prec = FP64 if dt == torch.float64 else FP32
        if outs is None:
            outs = [torch.empty_like(u) for u in us]
        _check(_lib.msb_group_apply(self._ptr, prec, self._ptrs(us, dt, "u"), self._ptrs(outs, dt, "f"), _stream()))
        return outs

    def autotune(self, precision: str = "fp64", effort: int = 1):
        """Time candidate group configurations (every member's products in one launch per
        pass) and keep the fastest.  Returns (configuration dict, group product ms)."""
        c = _LaunchConfig()
        ms = ctypes.c_double(0.0)
        _check(_lib.msb_group_autotune(self._ptr, _PREC[precision], int(effort), ctypes.byref(c), ctypes.byref(ms)))
        return {k: getattr(c, k) for k in CONFIG_KEYS}, ms.value

    def set_infl(self, infls, per_case=None):
        """New influence coefficients for every member in one call (msb_group_set_infl):
        infls[i] of shape (k,), or (B_i, k) where per_case[i] is true; the members' host
        work runs on parallel host threads."""
        n = len(self.plans)
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in infls]
        if len(arrs) != n:
            raise ValueError("one coefficient array per member (%d)" % n)
        pc = [bool(x) for x in (per_case if per_case is not None else [False] * n)]
        ks = {a.shape[-1] if a.ndim else 0 for a in arrs}
        if len(ks) != 1:
            raise ValueError("every member needs the same number of coefficients")
        k = ks.pop()
        for i, (a, p, c) in enumerate(zip(arrs, self.plans, pc)):
            if a.size != (p.batch if c else 1) * k:
                raise ValueError("member %d: expected %d coefficients" % (i, (p.batch if c else 1) * k))
        ptrs = (ctypes.c_void_p * n)(*[a.ctypes.data for a in arrs])
        flags = (ctypes.c_int * n)(*[int(c) for c in pc])
        _check(_lib.msb_group_set_infl(self._ptr, ptrs, int(k), flags))
        for p, a, c in zip(self.plans, arrs, pc):
            p.n_infl = int(k)
            p._infl_state = (a.copy(), c)

    def solve(self, bs, gs=None, precision: str = "fp64", tol: float = 1e-10, maxit: int = 100000,
              inner_tol: float = 0.0, graph_block=None, outs=None, check: bool = True, precond=None,
              reliable_update=None):
        """Static solves of every member at once; returns (list of u, list of per-member info lists).
        precond: each member's CG preconditioned by its circulant inverse; graph_block: CG
        iterations per hipGraph launch; reliable_update: FP32_REFINED keeps the search
        directions across residual replacements (None: the group's `precond` /
        `graph_block` / `reliable_update` attributes, which the autograd function's solves
        also use)."""
        torch = _torch()
        if outs is None:
            outs = [torch.empty_like(b) for b in bs]
        pre = self.precond if precond is None else bool(precond)
        gb = self.graph_block if graph_block is None else int(graph_block)
        rel = self.reliable_update if reliable_update is None else int(reliable_update)
        opts = _Opts(tol, int(maxit), float(inner_tol), gb, int(rel), int(pre))
        infos = (_Info * self.total_cases)()
        gp = None
        if gs is not None:
            gp = (ctypes.c_void_p * len(gs))(*[(p._vec(g, torch.float64, "g").value if g is not None else None)
                                               for p, g in zip(self.plans, gs)])
        st = _lib.msb_group_solve_static(self._ptr, _PREC[precision], self._ptrs(bs, torch.float64, "b"), gp,
                                         self._ptrs(outs, torch.float64, "u"), ctypes.byref(opts), infos, _stream())
        flat = [SolveInfo(i.status, i.outer_iters, i.inner_iters, i.rel_residual, i.seconds) for i in infos]
        res, k = [], 0
        for p in self.plans:
            res.append(flat[k:k + p.batch])
            k += p.batch
        if check:
            _check(st)
        return outs, res


def make_solve_function():
    """torch.autograd.Function for u = K(a)^{-1} b with the hand-written adjoint.

    forward(plan, b, infl[, precision, tol, precond]) -> u; backward: w = K^{-1} grad_u (K
    symmetric, same solve, same preconditioning),
    grad_b = w, grad_infl[b, k] = w . (A_k u)_F."""
    torch = _torch()

    class MSBFMSolve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, plan, b, infl, precision="fp32_refined", tol=1e-10, precond=False):
            plan.set_infl(infl.detach().cpu().numpy(), per_case=(infl.dim() == 2))
            u, _ = plan.solve(b.contiguous(), precision=precision, tol=tol, precond=precond)
            ctx.plan, ctx.precision, ctx.tol, ctx.precond = plan, precision, tol, precond
            ctx.per_case, ctx.infl_device = infl.dim() == 2, infl.device
            ctx.state = plan._operator_state()      # the operator this forward solve used
            ctx.save_for_backward(u)
            return u

        @staticmethod
        def backward(ctx, grad_u):
            (u,) = ctx.saved_tensors
            back = ctx.plan._restore_operator(ctx.state)
            try:
                w, _ = ctx.plan.solve(grad_u.contiguous(), precision=ctx.precision, tol=ctx.tol,
                                      precond=ctx.precond)
                ga = torch.from_numpy(ctx.plan.grad_infl(u, w))
            finally:
                if back is not None:
                    ctx.plan.set_infl(back[0], per_case=back[1])
            if not ctx.per_case:
                ga = ga.sum(0)          # one coefficient set shared by every case
            return None, w, ga.to(ctx.infl_device), None, None, None

    return MSBFMSolve


def make_group_solve_function():
    """torch.autograd.Function for u_i = K_i(a_i)^{-1} b_i over a PlanGroup, with the
    hand-written adjoint done as one group solve.

    apply(group, precision, tol, b_0..b_{n-1}, a_0..a_{n-1}) -> (u_0, ..., u_{n-1});
    backward: w_i = K_i^{-1} grad_u_i (all members in one group solve), grad_b_i = w_i,
    grad_a_i[b, k] = w_i . (A_{i,k} u_i)_F."""
    torch = _torch()

    class MSBFMGroupSolve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, group, precision, tol, *tensors):
            n = len(group.plans)
            bs, infls = tensors[:n], tensors[n:]
            group.set_infl([a.detach().cpu().numpy() for a in infls], per_case=[a.dim() == 2 for a in infls])
            us, _ = group.solve([b.contiguous() for b in bs], precision=precision, tol=tol)
            ctx.group, ctx.precision, ctx.tol = group, precision, tol
            ctx.per_case = [a.dim() == 2 for a in infls]
            ctx.devs = [a.device for a in infls]
            ctx.states = [p._operator_state() for p in group.plans]
            ctx.save_for_backward(*us)
            return tuple(us)

        @staticmethod
        def backward(ctx, *grad_us):
            us = ctx.saved_tensors
            gus = [torch.zeros_like(u) if g is None else g.contiguous() for u, g in zip(us, grad_us)]
            plans = ctx.group.plans
            for p, st in zip(plans, ctx.states):
                if st[2] != p._struct_version:
                    raise RuntimeError("a member's constraints, broken bonds or surface factors changed between "
                                       "the forward solve and its adjoint")
            changed = any(not (p._infl_state[1] == st[1] and p._infl_state[0].shape == st[0].shape
                               and np.array_equal(p._infl_state[0], st[0])) for p, st in zip(plans, ctx.states))
            back = [p._operator_state() for p in plans] if changed else None
            try:
                if changed:
                    ctx.group.set_infl([st[0] for st in ctx.states], per_case=[st[1] for st in ctx.states])
                ws, _ = ctx.group.solve(gus, precision=ctx.precision, tol=ctx.tol)
                gas = []
                for p, u, w, pc, dev in zip(plans, us, ws, ctx.per_case, ctx.devs):
                    ga = torch.from_numpy(p.grad_infl(u, w))
                    if not pc:
                        ga = ga.sum(0)
                    gas.append(ga.to(dev))
            finally:
                if back is not None:
                    ctx.group.set_infl([st[0] for st in back], per_case=[st[1] for st in back])
            return (None, None, None, *ws, *gas)

    return MSBFMGroupSolve
