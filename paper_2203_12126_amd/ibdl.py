"""Thin ctypes binding of ``libibdl.so`` (the C ABI in ``include/ibdl.h``).

Argument marshalling only: every step of the IBDL path runs in the HIP
library.  Torch tensors provide device memory and the current HIP stream.
If the library has not been built, every call raises ``RuntimeError``.
"""
from __future__ import annotations

import ctypes
import os
from collections.abc import Sequence
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibdl.so")

OK, ERR_ARG, ERR_OOM, ERR_HIP, ERR_NOCONV, ERR_NUMERIC, ERR_STATE = range(7)
DIRICHLET, NEUMANN = 0, 1
PESKIN4, COSINE4 = 0, 1
FP64, MIXED = 0, 1
LAP_FD, LAP_SPECTRAL = 0, 1
FORM_DOUBLE_LAYER, FORM_COMPLETED, FORM_SINGLE_LAYER = 0, 1, 2

_STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_OOM", 3: "ERR_HIP", 4: "ERR_NOCONV", 5: "ERR_NUMERIC",
           6: "ERR_STATE"}


class IbdlError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("lo", ctypes.c_double * 3),
                ("length", ctypes.c_double), ("alpha", ctypes.c_double), ("bc", ctypes.c_int32),
                ("delta", ctypes.c_int32), ("prec", ctypes.c_int32), ("npts", ctypes.c_int32),
                ("X", ctypes.c_void_p), ("normal", ctypes.c_void_p), ("weight", ctypes.c_void_p),
                ("lap", ctypes.c_int32), ("form", ctypes.c_int32), ("eta", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("x0", ctypes.c_void_p), ("true_residual", ctypes.c_int32)]


class PlanStats(ctypes.Structure):
    _fields_ = [("nlines", ctypes.c_int32), ("pitch", ctypes.c_int32),
                ("n_spread_lines", ctypes.c_int32), ("n_gather_lines", ctypes.c_int32),
                ("n_spread_planes", ctypes.c_int32), ("n_gather_planes", ctypes.c_int32),
                ("dip_active_nodes", ctypes.c_int32), ("dip_nnz", ctypes.c_int64),
                ("mono_nnz", ctypes.c_int64), ("col_tile", ctypes.c_int32), ("z_rows", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("rel_resid_est", ctypes.c_double),
                ("rel_resid_true", ctypes.c_double), ("status", ctypes.c_int32),
                ("fp64_applies", ctypes.c_int32)]


class RequestTimes(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("cohort_size", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("cohorts", ctypes.c_int64),
                ("pending", ctypes.c_int32), ("active", ctypes.c_int32), ("peak_active", ctypes.c_int32),
                ("in_use_bytes", ctypes.c_size_t), ("peak_in_use_bytes", ctypes.c_size_t),
                ("budget_bytes", ctypes.c_size_t)]


_lib = None


def lib():
    """Load libibdl.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int32
    st = ctypes.c_int
    sig = {
        "ibdl_plan_create": ([ctypes.POINTER(Desc), P, ctypes.POINTER(P)], st),
        "ibdl_plan_destroy": ([P], st),
        "ibdl_plan_footprint": ([ctypes.POINTER(Desc), I, I], ctypes.c_size_t),
        "ibdl_apply": ([P, I, P, P, P], st),
        "ibdl_apply_noalloc": ([P, I, P, P, P], st),
        "ibdl_rhs": ([P, I, P, P, P, P], st),
        "ibdl_solve": ([P, I, P, P, ctypes.POINTER(SolveOpts), P, ctypes.POINTER(SolveInfo), P], st),
        "ibdl_solve_grid": ([P, I, P, P, ctypes.POINTER(SolveOpts), P, P, ctypes.POINTER(SolveInfo), P], st),
        "ibdl_eval_grid": ([P, I, P, P, P, P, P], st),
        "ibdl_plan_binning": ([P, P, P], st),
        "ibdl_indicator": ([P, P, P, P], st),
        "ibdl_fixup": ([P, I, P, P, P, ctypes.c_double, ctypes.c_double, P, P], st),
        "ibdl_plan_set_timing": ([P, I], st),
        "ibdl_plan_stage_times": ([P, P, P, P, I, ctypes.POINTER(I)], st),
        "ibdl_plan_get_stats": ([P, ctypes.POINTER(PlanStats)], st),
        "ibdl_last_error": ([], ctypes.c_char_p),
        "ibdl_batch_create": ([ctypes.POINTER(Desc), I, P, P, ctypes.POINTER(P)], st),
        "ibdl_batch_destroy": ([P], st),
        "ibdl_batch_size": ([P, ctypes.POINTER(I), ctypes.POINTER(I)], st),
        "ibdl_batch_apply": ([P, P, P, P], st),
        "ibdl_batch_get_stats": ([P, I, ctypes.POINTER(PlanStats)], st),
        "ibdl_batch_solve": ([P, P, P, ctypes.POINTER(SolveOpts), P, ctypes.POINTER(SolveInfo), P], st),
        "ibdl_batch_solve_grid": ([P, P, P, ctypes.POINTER(SolveOpts), P, P, ctypes.POINTER(SolveInfo), P], st),
        "ibdl_batch_eval_grid": ([P, P, P, P, P, P], st),
        "ibdl_batch_set_timing": ([P, I], st),
        "ibdl_batch_stage_times": ([P, P, P, P, I, ctypes.POINTER(I)], st),
        "ibdl_server_create": ([ctypes.c_size_t, I, I, ctypes.POINTER(P)], st),
        "ibdl_server_destroy": ([P], st),
        "ibdl_server_footprint": ([ctypes.POINTER(Desc), I, I, ctypes.POINTER(ctypes.c_size_t)], st),
        "ibdl_server_submit": ([P, ctypes.POINTER(Desc), I, P, P, ctypes.POINTER(SolveOpts), P, P, P,
                                ctypes.POINTER(ctypes.c_uint64)], st),
        "ibdl_server_poll": ([P, ctypes.c_uint64, ctypes.POINTER(SolveInfo), ctypes.POINTER(RequestTimes)], st),
        "ibdl_server_wait": ([P, ctypes.c_uint64, ctypes.POINTER(SolveInfo), ctypes.POINTER(RequestTimes)], st),
        "ibdl_server_get_stats": ([P, ctypes.POINTER(ServerStats)], st),
        "ibdl_set_autotune": ([I], st),
        "ibdl_set_graphs": ([I], st),
        "ibdl_graph_stats": ([ctypes.c_void_p], st),
        "ibdl_autotune_report": ([ctypes.c_char_p, ctypes.c_size_t], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def last_error() -> str:
    return lib().ibdl_last_error().decode()


def _check(status: int, what: str):
    if status != OK:
        raise IbdlError(status, f"{what}: {last_error()}")


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _bptr(t, name, shape):
    """A contiguous uint8 CUDA tensor of `shape` elements as a device pointer."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous uint8 CUDA tensor")
    if t.numel() != shape:
        raise ValueError(f"{name} has {t.numel()} elements, expected {shape}")
    return ctypes.c_void_p(t.data_ptr())


def _dptr(t, name, shape=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and t.numel() != shape:
        raise ValueError(f"{name} has {t.numel()} elements, expected {shape}")
    return ctypes.c_void_p(t.data_ptr())


def make_desc(dim, n, lo, length, alpha, bc, delta, prec, npts, X=None, normal=None, weight=None, lap=0, form=0,
              eta=0.0):
    d = Desc()
    d.dim, d.n = dim, n
    for i in range(3):
        d.lo[i] = float(lo[i]) if i < len(lo) else 0.0
    d.length, d.alpha = float(length), float(alpha)
    d.bc, d.delta, d.prec, d.npts = bc, delta, prec, npts
    d.X = X.data_ptr() if X is not None else None
    d.normal = normal.data_ptr() if normal is not None else None
    d.weight = weight.data_ptr() if weight is not None else None
    d.lap = lap
    d.form = form
    d.eta = float(eta)
    return d


def set_autotune(enable: bool = True, force=None):
    """Clear the tile autotuner's choices and turn it on or off; force=v (0..3)
    uses row-block shape v everywhere (for tests)."""
    mode = 2 + int(force) if force is not None else (1 if enable else 0)
    _check(lib().ibdl_set_autotune(mode), "ibdl_set_autotune")


def set_graphs(enable: bool = True):
    """Replay each GMRES-Arnoldi step from a recorded HIP graph, or launch its
    kernels one by one (the default); results are bit-identical."""
    _check(lib().ibdl_set_graphs(1 if enable else 0), "ibdl_set_graphs")


def graph_stats() -> dict:
    """Process totals: graphs recorded and step replays."""
    out = (ctypes.c_int64 * 2)()
    _check(lib().ibdl_graph_stats(out), "ibdl_graph_stats")
    return {"recorded": out[0], "replays": out[1]}


def autotune_report() -> str:
    n = lib().ibdl_autotune_report(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib().ibdl_autotune_report(buf, n + 1)
    return buf.value.decode()


def footprint(dim, n, npts, bc=DIRICHLET, prec=FP64, nrhs=1, restart=50) -> int:
    """Device bytes of a plan plus solve workspace (host-only estimate)."""
    d = make_desc(dim, n, (0, 0, 0), 1.0, 1.0, bc, PESKIN4, prec, npts)
    d.X = d.normal = d.weight = 1  # non-null placeholders: the estimate never dereferences them
    return int(lib().ibdl_plan_footprint(ctypes.byref(d), nrhs, restart))


class Plan:
    """One geometry on one periodic grid (``ibdl_plan``)."""

    def __init__(self, dim, n, lo, length, alpha, X, normal, weight, bc=DIRICHLET, delta=PESKIN4,
                 prec=FP64, stream=None, lap=0, form=0, eta=0.0):
        import torch
        self._keep = [t.contiguous() for t in (X, normal, weight)]
        X, normal, weight = self._keep
        m = int(weight.numel())
        _dptr(X, "X", m * dim)
        _dptr(normal, "normal", m * dim)
        _dptr(weight, "weight", m)
        self.dim, self.n, self.m, self.bc, self.prec = dim, n, m, bc, prec
        self.form = form
        # unknowns per right-hand side: M, or M + 1 for the completed formulation ([Q; ubar])
        self.nu = m + 1 if form == FORM_COMPLETED else m
        self.grid_size = n ** dim
        d = make_desc(dim, n, lo, length, alpha, bc, delta, prec, m, X, normal, weight, lap=lap, form=form, eta=eta)
        h = ctypes.c_void_p()
        _check(lib().ibdl_plan_create(ctypes.byref(d), _stream(stream), ctypes.byref(h)),
               "ibdl_plan_create")
        self._h = h
        self._keep = None
        self._torch = torch

    @classmethod
    def from_problem(cls, prob, delta=PESKIN4, prec=FP64, device="cuda", lap=0, form=0, eta=0.0):
        import torch
        g = prob.grid
        t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device).contiguous()
        return cls(g.dim, g.n, tuple(g.lo), g.length, prob.alpha, t(prob.geom.X), t(prob.geom.normal),
                   t(prob.geom.weight), bc=prob.bc, delta=delta, prec=prec, lap=lap, form=form, eta=eta)

    # ------------------------------------------------------------------
    def _empty(self, *shape):
        return self._torch.empty(*shape, dtype=self._torch.float64, device="cuda")

    def _nrhs(self, t, per):
        if t.numel() % per:
            raise ValueError("array size is not a multiple of the per-rhs size")
        return t.numel() // per

    def apply(self, q, out=None, stream=None):
        nrhs = self._nrhs(q, self.nu)
        out = self._empty(*q.shape) if out is None else out
        _check(lib().ibdl_apply(self._h, nrhs, _dptr(q, "q"), _dptr(out, "Aq", q.numel()),
                                _stream(stream)), "ibdl_apply")
        return out

    def apply_noalloc(self, q, out, stream=None):
        """ibdl_apply_noalloc: the operator with the library's fixed device scratch
        (no device allocation; out must be given)."""
        nrhs = self._nrhs(q, self.m)
        _check(lib().ibdl_apply_noalloc(self._h, nrhs, _dptr(q, "q"), _dptr(out, "Aq", q.numel()),
                                        _stream(stream)), "ibdl_apply_noalloc")
        return out

    def rhs(self, data, g=None, out=None, stream=None):
        nrhs = self._nrhs(data, self.m)
        out = self._empty(nrhs, self.nu) if out is None else out
        _check(lib().ibdl_rhs(self._h, nrhs, _dptr(data, "data"),
                              _dptr(g, "g", nrhs * self.grid_size), _dptr(out, "b", nrhs * self.nu),
                              _stream(stream)), "ibdl_rhs")
        return out

    def solve(self, data, g=None, tol=1e-8, restart=50, maxit=500, x0=None, true_residual=False,
              out=None, stream=None, raise_on_noconv=True):
        nrhs = self._nrhs(data, self.m)
        out = self._empty(nrhs, self.nu) if out is None else out
        o = SolveOpts(tol, restart, maxit, None, 1 if true_residual else 0)
        if x0 is not None:
            o.x0 = _dptr(x0, "x0", data.numel()).value
        info = (SolveInfo * nrhs)()
        st = lib().ibdl_solve(self._h, nrhs, _dptr(data, "data"), _dptr(g, "g", nrhs * self.grid_size),
                              ctypes.byref(o), _dptr(out, "sol", nrhs * self.nu), info, _stream(stream))
        if st != OK and not (st == ERR_NOCONV and not raise_on_noconv):
            _check(st, "ibdl_solve")
        return out, InfoList(info)

    def solve_grid(self, data, g=None, tol=1e-8, restart=50, maxit=500, x0=None, true_residual=False,
                   out=None, u=None, stream=None, raise_on_noconv=True):
        """solve() and the grid solution (V_b = data for Neumann) in one call."""
        nrhs = self._nrhs(data, self.m)
        out = self._empty(nrhs, self.nu) if out is None else out
        u = self._empty(nrhs, *([self.n] * self.dim)) if u is None else u
        o = SolveOpts(tol, restart, maxit, None, 1 if true_residual else 0)
        if x0 is not None:
            o.x0 = _dptr(x0, "x0", data.numel()).value
        info = (SolveInfo * nrhs)()
        st = lib().ibdl_solve_grid(self._h, nrhs, _dptr(data, "data"), _dptr(g, "g", nrhs * self.grid_size),
                                   ctypes.byref(o), _dptr(out, "sol", nrhs * self.nu),
                                   _dptr(u, "u", nrhs * self.grid_size), info, _stream(stream))
        if st != OK and not (st == ERR_NOCONV and not raise_on_noconv):
            _check(st, "ibdl_solve_grid")
        return out, u, InfoList(info)

    def eval_grid(self, sol, vb=None, g=None, out=None, stream=None):
        nrhs = self._nrhs(sol, self.nu)
        out = self._empty(nrhs, *([self.n] * self.dim)) if out is None else out
        _check(lib().ibdl_eval_grid(self._h, nrhs, _dptr(sol, "sol"), _dptr(vb, "vb", nrhs * self.m),
                                    _dptr(g, "g", nrhs * self.grid_size),
                                    _dptr(out, "u", nrhs * self.grid_size), _stream(stream)),
               "ibdl_eval_grid")
        return out

    def indicator(self, stream=None):
        """ibdl_indicator: (chi, flags) on the grid (App. D)."""
        import torch
        chi = self._empty(*([self.n] * self.dim))
        flags = torch.empty(*([self.n] * self.dim), dtype=torch.uint8, device="cuda")
        _check(lib().ibdl_indicator(self._h, _dptr(chi, "chi", self.grid_size), _bptr(flags, "flags", self.grid_size),
                                    _stream(stream)), "ibdl_indicator")
        return chi, flags

    def fixup(self, u, ub, flags, m1=6.0, m2=8.0, out=None, stream=None):
        """ibdl_fixup: the near-boundary re-interpolation of App. A."""
        nrhs = self._nrhs(u, self.grid_size)
        out = self._empty(*u.shape) if out is None else out
        _check(lib().ibdl_fixup(self._h, nrhs, _dptr(u, "u"), _dptr(ub, "ub", nrhs * self.m),
                                _bptr(flags, "flags", self.grid_size),
                                float(m1), float(m2), _dptr(out, "u_out", u.numel()), _stream(stream)),
               "ibdl_fixup")
        return out

    def binning(self):
        import numpy as np
        key = np.zeros(self.m, dtype=np.uint32)
        perm = np.zeros(self.m, dtype=np.uint32)
        _check(lib().ibdl_plan_binning(self._h, key.ctypes.data_as(ctypes.c_void_p),
                                       perm.ctypes.data_as(ctypes.c_void_p)), "ibdl_plan_binning")
        return key, perm

    def stats(self) -> dict:
        s = PlanStats()
        _check(lib().ibdl_plan_get_stats(self._h, ctypes.byref(s)), "ibdl_plan_get_stats")
        return {f: getattr(s, f) for f, _ in PlanStats._fields_}

    def set_timing(self, on=True):
        _check(lib().ibdl_plan_set_timing(self._h, 1 if on else 0), "ibdl_plan_set_timing")

    def stage_times(self):
        """[(stage name, mean ms, timed calls)] since timing was enabled."""
        ms = (ctypes.c_double * 16)()
        names = (ctypes.c_char_p * 16)()
        calls = (ctypes.c_int64 * 16)()
        cnt = ctypes.c_int32()
        _check(lib().ibdl_plan_stage_times(self._h, ms, names, calls, 16, ctypes.byref(cnt)),
               "ibdl_plan_stage_times")
        return [(names[i].decode(), ms[i], calls[i]) for i in range(cnt.value)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ibdl_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class InfoList(Sequence):
    """Per-rhs solve reports over the C array the library filled: item r is a dict
    (iters, rel_resid_est, rel_resid_true, status, fp64_applies), built when it is
    read; field(name) returns one of them for every rhs as a numpy array."""

    _keys = tuple(f for f, _ in SolveInfo._fields_)

    def __init__(self, info):
        import numpy as np
        f = SolveInfo._fields_
        dt = np.dtype(dict(names=[n for n, _ in f],
                           formats=["<i4" if t is ctypes.c_int32 else "<f8" for _, t in f],
                           offsets=[getattr(SolveInfo, n).offset for n, _ in f],
                           itemsize=ctypes.sizeof(SolveInfo)))
        self._a = np.frombuffer(info, dtype=dt)

    def __len__(self):
        return len(self._a)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[j] for j in range(*i.indices(len(self._a)))]
        rec = self._a[i]
        return {k: rec[k].item() for k in self._keys}

    def field(self, name):
        return self._a[name].copy()

    def __repr__(self):
        return repr(list(self))


def _ptr_array(tensors, name, sizes, allow_none=False):
    """Host array of device pointers, one per instance (None entries -> NULL)."""
    import torch
    f64, tensor = torch.float64, torch.Tensor
    ptrs = [None] * len(tensors)
    for i, t in enumerate(tensors):
        if t is None:
            if not allow_none:
                raise ValueError(f"{name}[{i}] is required")
            continue
        if not isinstance(t, tensor) or t.dtype is not f64 or not t.is_cuda:
            raise TypeError(f"{name}[{i}] must be a float64 CUDA tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name}[{i}] must be contiguous")
        if sizes is not None and t.numel() != sizes[i]:
            raise ValueError(f"{name}[{i}] has {t.numel()} elements, expected {sizes[i]}")
        ptrs[i] = t.data_ptr()
    return (ctypes.c_void_p * len(ptrs))(*ptrs)


class Batch:
    """Many independent instances solved together (``ibdl_batch``).

    ``instances``: list of dicts with keys dim, n, lo, length, alpha, X, normal,
    weight (float64 CUDA tensors), bc, prec, nrhs and optionally delta."""

    def __init__(self, instances, stream=None):
        import torch
        self._torch = torch
        keep = []
        descs = (Desc * len(instances))()
        nrhs = (ctypes.c_int32 * len(instances))()
        self.meta = []
        for i, ins in enumerate(instances):
            X, nrm, w = (ins[k].contiguous() for k in ("X", "normal", "weight"))
            keep += [X, nrm, w]
            m = int(w.numel())
            dim, n = ins["dim"], ins["n"]
            _dptr(X, "X", m * dim)
            _dptr(nrm, "normal", m * dim)
            _dptr(w, "weight", m)
            descs[i] = make_desc(dim, n, ins.get("lo", (0.0, 0.0, 0.0)), ins.get("length", 1.0),
                                 ins["alpha"], ins.get("bc", DIRICHLET), ins.get("delta", PESKIN4),
                                 ins.get("prec", MIXED), m, X, nrm, w, lap=ins.get("lap", 0))
            nrhs[i] = int(ins["nrhs"])
            self.meta.append(dict(dim=dim, n=n, m=m, nrhs=int(ins["nrhs"]), bc=ins.get("bc", DIRICHLET)))
        h = ctypes.c_void_p()
        _check(lib().ibdl_batch_create(descs, len(instances), nrhs, _stream(stream), ctypes.byref(h)),
               "ibdl_batch_create")
        self._h = h
        self.count = len(instances)
        self.total_rhs = sum(mt["nrhs"] for mt in self.meta)

    @classmethod
    def from_problems(cls, items, prec=MIXED, delta=PESKIN4, device="cuda"):
        """items: list of (Problem, nrhs); geometry, grid, alpha and bc come from the Problem."""
        import torch
        t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device).contiguous()
        inst = []
        for prob, nrhs in items:
            g = prob.grid
            inst.append(dict(dim=g.dim, n=g.n, lo=tuple(g.lo), length=g.length, alpha=prob.alpha,
                             X=t(prob.geom.X), normal=t(prob.geom.normal), weight=t(prob.geom.weight),
                             bc=prob.bc, prec=prec, delta=delta, nrhs=nrhs))
        return cls(inst)

    def _sizes(self, grid=False):
        cache = self.__dict__.setdefault("_size_cache", {})
        if grid not in cache:
            cache[grid] = [mt["nrhs"] * (mt["n"] ** mt["dim"] if grid else mt["m"]) for mt in self.meta]
        return cache[grid]

    def empty(self, grid=False):
        """Uninitialised output tensors, one per instance: solutions [nrhs, M] or,
        with grid=True, grid solutions [nrhs, n, ...] (to pass as out= / u=)."""
        return self._empty_like_sizes(grid)

    def _empty_like_sizes(self, grid=False):
        out = []
        for mt in self.meta:
            shape = (mt["nrhs"], *([mt["n"]] * mt["dim"])) if grid else (mt["nrhs"], mt["m"])
            out.append(self._torch.empty(*shape, dtype=self._torch.float64, device="cuda"))
        return out

    def apply(self, q, out=None, stream=None):
        out = self._empty_like_sizes() if out is None else out
        _check(lib().ibdl_batch_apply(self._h, _ptr_array(q, "q", self._sizes()),
                                      _ptr_array(out, "Aq", self._sizes()), _stream(stream)),
               "ibdl_batch_apply")
        return out

    def solve(self, data, g=None, tol=1e-8, restart=50, maxit=500, true_residual=False, out=None,
              stream=None, raise_on_noconv=True):
        out = self._empty_like_sizes() if out is None else out
        o = SolveOpts(tol, restart, maxit, None, 1 if true_residual else 0)
        info = (SolveInfo * self.total_rhs)()
        garr = None if g is None else _ptr_array(g, "g", self._sizes(grid=True), allow_none=True)
        st = lib().ibdl_batch_solve(self._h, _ptr_array(data, "data", self._sizes()), garr, ctypes.byref(o),
                                    _ptr_array(out, "sol", self._sizes()), info, _stream(stream))
        if st != OK and not (st == ERR_NOCONV and not raise_on_noconv):
            _check(st, "ibdl_batch_solve")
        return out, InfoList(info)

    def solve_grid(self, data, g=None, tol=1e-8, restart=50, maxit=500, true_residual=False, out=None,
                   u=None, stream=None, raise_on_noconv=True):
        """solve() and every instance's grid solution (V_b = data for Neumann)."""
        out = self._empty_like_sizes() if out is None else out
        u = self._empty_like_sizes(grid=True) if u is None else u
        o = SolveOpts(tol, restart, maxit, None, 1 if true_residual else 0)
        info = (SolveInfo * self.total_rhs)()
        garr = None if g is None else _ptr_array(g, "g", self._sizes(grid=True), allow_none=True)
        st = lib().ibdl_batch_solve_grid(self._h, _ptr_array(data, "data", self._sizes()), garr, ctypes.byref(o),
                                         _ptr_array(out, "sol", self._sizes()),
                                         _ptr_array(u, "u", self._sizes(grid=True)), info, _stream(stream))
        if st != OK and not (st == ERR_NOCONV and not raise_on_noconv):
            _check(st, "ibdl_batch_solve_grid")
        return out, u, InfoList(info)

    def eval_grid(self, sol, vb=None, g=None, out=None, stream=None):
        out = self._empty_like_sizes(grid=True) if out is None else out
        vbarr = None if vb is None else _ptr_array(vb, "vb", self._sizes(), allow_none=True)
        garr = None if g is None else _ptr_array(g, "g", self._sizes(grid=True), allow_none=True)
        _check(lib().ibdl_batch_eval_grid(self._h, _ptr_array(sol, "sol", self._sizes()), vbarr, garr,
                                          _ptr_array(out, "u", self._sizes(grid=True)), _stream(stream)),
               "ibdl_batch_eval_grid")
        return out

    def stats(self, i) -> dict:
        s = PlanStats()
        _check(lib().ibdl_batch_get_stats(self._h, i, ctypes.byref(s)), "ibdl_batch_get_stats")
        return {f: getattr(s, f) for f, _ in PlanStats._fields_}

    def set_timing(self, on=True):
        _check(lib().ibdl_batch_set_timing(self._h, 1 if on else 0), "ibdl_batch_set_timing")

    def stage_times(self):
        ms = (ctypes.c_double * 16)()
        names = (ctypes.c_char_p * 16)()
        calls = (ctypes.c_int64 * 16)()
        cnt = ctypes.c_int32()
        _check(lib().ibdl_batch_stage_times(self._h, ms, names, calls, 16, ctypes.byref(cnt)),
               "ibdl_batch_stage_times")
        return [(names[i].decode(), ms[i], calls[i]) for i in range(cnt.value)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ibdl_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop (``ibdl_server``): submit solves, poll or wait for results.

    A request is a Problem-like set of tensors; the server keeps references to
    every tensor of a request until its result has been taken."""

    def __init__(self, budget_bytes=0, max_slots=64, streams=4):
        h = ctypes.c_void_p()
        _check(lib().ibdl_server_create(int(budget_bytes), int(max_slots), int(streams), ctypes.byref(h)),
               "ibdl_server_create")
        self._h = h
        self._req = {}

    @staticmethod
    def footprint(dim, n, npts, bc=DIRICHLET, prec=MIXED, nrhs=1, restart=50) -> int:
        d = make_desc(dim, n, (0, 0, 0), 1.0, 1.0, bc, PESKIN4, prec, npts)
        d.X = d.normal = d.weight = 1  # placeholders: the estimate never dereferences them
        out = ctypes.c_size_t()
        _check(lib().ibdl_server_footprint(ctypes.byref(d), nrhs, restart, ctypes.byref(out)),
               "ibdl_server_footprint")
        return int(out.value)

    def submit(self, dim, n, lo, length, alpha, X, normal, weight, data, g=None, bc=DIRICHLET,
               delta=PESKIN4, prec=MIXED, tol=1e-8, restart=50, maxit=500, grid=True, true_residual=False,
               stream=None, lap=0):
        """Queue one solve; returns a ticket.  data: (nrhs, M); g: (nrhs, n^dim) or None."""
        import torch
        m = int(weight.numel())
        nrhs = data.numel() // m
        _dptr(X, "X", m * dim)
        _dptr(normal, "normal", m * dim)
        _dptr(weight, "weight", m)
        sol = torch.empty(nrhs, m, dtype=torch.float64, device="cuda")
        u = torch.empty(nrhs, *([n] * dim), dtype=torch.float64, device="cuda") if grid else None
        d = make_desc(dim, n, lo, length, alpha, bc, delta, prec, m, X, normal, weight, lap=lap)
        o = SolveOpts(tol, restart, maxit, None, 1 if true_residual else 0)
        t = ctypes.c_uint64()
        _check(lib().ibdl_server_submit(self._h, ctypes.byref(d), nrhs, _dptr(data, "data", nrhs * m),
                                        _dptr(g, "g", nrhs * n ** dim), ctypes.byref(o), _dptr(sol, "sol"),
                                        _dptr(u, "u") if u is not None else None, _stream(stream),
                                        ctypes.byref(t)), "ibdl_server_submit")
        self._req[t.value] = dict(keep=(X, normal, weight, data, g), sol=sol, u=u, nrhs=nrhs)
        return t.value

    def submit_problem(self, prob, nrhs_data=None, prec=MIXED, **kw):
        import torch
        g = prob.grid
        T = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
        data = T(prob.data).reshape(1, -1) if nrhs_data is None else T(nrhs_data[0])
        gt = T(prob.g_tilde).reshape(1, -1) if nrhs_data is None else T(nrhs_data[1])
        return self.submit(g.dim, g.n, tuple(g.lo), g.length, prob.alpha, T(prob.geom.X), T(prob.geom.normal),
                           T(prob.geom.weight), data, gt, bc=prob.bc, prec=prec, **kw)

    def _result(self, fn, ticket, raise_on_error):
        rq = self._req[ticket]
        info = (SolveInfo * rq["nrhs"])()
        tm = RequestTimes()
        st = fn(self._h, ticket, info, ctypes.byref(tm))
        if st == ERR_STATE:
            return None
        del self._req[ticket]
        if st != OK and raise_on_error and st != ERR_NOCONV:
            _check(st, "request")
        return dict(status=st, sol=rq["sol"], u=rq["u"], info=InfoList(info),
                    times=dict(queue_ms=tm.queue_ms, run_ms=tm.run_ms, total_ms=tm.total_ms,
                               cohort_size=tm.cohort_size))

    def poll(self, ticket, raise_on_error=True):
        """None while pending, else dict(status, sol, u, info, times)."""
        return self._result(lib().ibdl_server_poll, ticket, raise_on_error)

    def wait(self, ticket, raise_on_error=True):
        return self._result(lib().ibdl_server_wait, ticket, raise_on_error)

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().ibdl_server_get_stats(self._h, ctypes.byref(s)), "ibdl_server_get_stats")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ibdl_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
