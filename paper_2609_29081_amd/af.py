"""Thin ctypes binding of libaf.so (include/af.h).

Argument marshalling only: every step of the method runs in the HIP
library.  torch provides device memory and streams.  Importing this module
fails loudly if the built library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaf.so")

AF_OK, AF_E_ARG, AF_E_HIP, AF_E_PP, AF_E_NONFINITE = 0, 1, 2, 3, 4
PERIODIC, OUTFLOW, NOSLIP, SYMMETRY, DIRICHLET = 0, 1, 2, 3, 4
LIM_SMOOTH, LIM_PP, LIM_POINT, LIM_CENTRE, LIM_LOWONLY, LIM_LEARNED = 1, 2, 4, 8, 16, 32
LIM_PEXACT = 64   # theta^p by the root of the pressure quadratic
LIM_ALL = 15
PREC_FP64, PREC_MIXED = 0, 1
FLAG_CELL_LOW, FLAG_POINT_LOW, FLAG_NONFINITE = 1, 2, 4


class AFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"af status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("dim", C.c_int), ("n1", C.c_int), ("n2", C.c_int),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("gamma", C.c_double), ("mu", C.c_double), ("Pr", C.c_double),
                ("cfl_c", C.c_double), ("cfl_v", C.c_double), ("Cs", C.c_double),
                ("limiter", C.c_int), ("max_halvings", C.c_int), ("precision", C.c_int),
                ("rk", C.c_int)]


_lib = None

EXPORTS = ["af_default_params", "af_init_grid", "af_destroy", "af_set_bc", "af_set_bc_state",
           "af_state_len",
           "af_state_bytes", "af_workspace_bytes", "af_set_state", "af_get_state",
           "af_check_admissible", "af_rk_stage", "af_cfl_dt", "af_step", "af_run",
           "af_read_flags", "af_reset_flags", "af_timing", "af_timing_read", "af_last_error",
           "af_batch_create", "af_batch_destroy", "af_batch_workspace_bytes", "af_batch_run",
           "af_stage_variant_count", "af_stage_variant_info", "af_batch_variant",
           "af_batch_set_variant", "af_batch_tune", "af_face_count", "af_mlp_param_count",
           "af_blend_features", "af_set_blend_net", "af_blend_infer", "af_rk_stage_blend",
           "af_mlp_grad_workspace_bytes", "af_mlp_grad", "af_mlp_adam", "af_mlp_train",
           "af_stage_times", "af_step_source", "af_step_noalloc", "af_run_graph"]

# kernel kinds reported by af_timing_read
KERNEL_KINDS = {0: "lattice", 1: "grad", 2: "cellpre", 3: "face", 4: "cells", 5: "points",
                6: "cfl", 7: "stage2d", 8: "blend"}
K_COUNT = 9


def lib():
    """load libaf.so (raises if it has not been built)"""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built: run __graft_entry__.build() "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.c_int
        L.af_default_params.argtypes = [C.POINTER(Params)]
        L.af_init_grid.argtypes = [C.POINTER(Params), C.POINTER(vp)]
        L.af_destroy.argtypes = [vp]
        L.af_destroy.restype = None
        L.af_set_bc.argtypes = [vp, ip, ip]
        L.af_set_bc_state.argtypes = [vp, ip, dp]
        L.af_state_len.argtypes = [vp]
        L.af_state_len.restype = C.c_size_t
        L.af_workspace_bytes.argtypes = [vp]
        L.af_workspace_bytes.restype = C.c_size_t
        L.af_state_bytes.argtypes = [vp]
        L.af_state_bytes.restype = C.c_size_t
        L.af_set_state.argtypes = [vp, vp, vp, vp]
        L.af_get_state.argtypes = [vp, vp, vp, vp]
        L.af_check_admissible.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_long)]
        L.af_batch_create.argtypes = [C.POINTER(vp), ip, C.POINTER(vp)]
        L.af_batch_destroy.argtypes = [vp]
        L.af_batch_destroy.restype = None
        L.af_batch_workspace_bytes.argtypes = [vp]
        L.af_batch_workspace_bytes.restype = C.c_size_t
        fp = C.POINTER(C.c_float)
        L.af_face_count.argtypes = [vp]
        L.af_face_count.restype = C.c_long
        L.af_mlp_param_count.argtypes = []
        L.af_mlp_param_count.restype = C.c_size_t
        L.af_blend_features.argtypes = [vp, vp, vp, vp]
        L.af_set_blend_net.argtypes = [vp, vp]
        L.af_blend_infer.argtypes = [vp, vp, vp, vp, vp]
        L.af_rk_stage_blend.argtypes = [vp, ip, vp, C.c_double, vp, vp, vp, vp, vp, vp, vp]
        L.af_mlp_grad_workspace_bytes.argtypes = [C.c_long]
        L.af_mlp_grad_workspace_bytes.restype = C.c_size_t
        L.af_mlp_grad.argtypes = [vp, vp, C.c_long, vp, vp, vp, vp, vp]
        L.af_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_long, C.c_float, vp]
        L.af_mlp_train.argtypes = [vp, vp, C.c_long, vp, vp, vp, vp, C.c_long, ip, ip, C.c_float,
                                   vp, vp, vp]
        L.af_stage_times.argtypes = [ip, dp]
        L.af_step_source.argtypes = [vp, vp, vp, vp, C.c_double, C.POINTER(vp), ip]
        L.af_stage_variant_count.argtypes = []
        L.af_stage_variant_info.argtypes = [ip, C.POINTER(C.c_char_p), C.POINTER(ip),
                                            C.POINTER(ip)]
        L.af_batch_variant.argtypes = [vp]
        L.af_batch_set_variant.argtypes = [vp, ip]
        L.af_batch_tune.argtypes = [vp, C.POINTER(vp), vp, vp, C.c_double, C.c_double, ip, dp]
        L.af_batch_run.argtypes = [vp, C.POINTER(vp), vp, vp, C.c_double, C.c_double, C.c_long, ip,
                                   ip, C.POINTER(C.c_long), dp, C.POINTER(C.c_int),
                                   C.POINTER(C.c_long)]
        L.af_rk_stage.argtypes = [vp, ip, vp, C.c_double, vp, vp, vp, vp, vp]
        L.af_cfl_dt.argtypes = [vp, vp, C.c_double, C.c_double, vp, vp, vp]
        L.af_step.argtypes = [vp, vp, vp, vp, C.c_double, C.c_double, C.c_double, dp,
                              C.POINTER(C.c_int)]
        L.af_step_noalloc.argtypes = [vp, vp, vp, C.c_double, C.c_double, C.c_double, dp,
                                      C.POINTER(C.c_int)]
        L.af_run.argtypes = [vp, vp, vp, vp, C.c_double, C.c_double, C.c_long, ip,
                             C.POINTER(C.c_long), dp]
        L.af_run_graph.argtypes = [vp, vp, vp, vp, C.c_double, C.c_double, C.c_long, ip,
                                   C.POINTER(C.c_long), dp, C.POINTER(C.c_long)]
        L.af_read_flags.argtypes = [vp, vp, C.POINTER(C.c_int), vp]
        L.af_reset_flags.argtypes = [vp, vp, vp]
        L.af_timing.argtypes = [vp, ip]
        L.af_timing_read.argtypes = [vp, C.POINTER(C.c_long), dp]
        L.af_last_error.restype = C.c_char_p
        for name in ("af_default_params", "af_init_grid", "af_set_bc", "af_rk_stage", "af_cfl_dt",
                     "af_step", "af_step_noalloc", "af_run", "af_run_graph", "af_read_flags", "af_reset_flags", "af_timing",
                     "af_timing_read"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != AF_OK:
        raise AFError(st, lib().af_last_error().decode())


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Solver:
    """One grid: wraps af_init_grid / af_set_bc and owns the torch-allocated
    workspace.  States are flat float64 CUDA tensors of length state_len."""

    def __init__(self, grid: W.Grid, gamma=1.4, mu=1e-3, Pr=0.72, cfl_c=0.2, cfl_v=0.05,
                 limiter=LIM_ALL, Cs=1.0, max_halvings=40, precision=0, rk=3, bcstate=None,
                 device="cuda:0"):
        p = Params()
        _check(lib().af_default_params(C.byref(p)))
        p.dim, p.n1, p.n2 = grid.dim, grid.n1, grid.n2
        p.x0, p.x1, p.y0, p.y1 = grid.x0, grid.x1, grid.y0, grid.y1
        p.gamma, p.mu, p.Pr = gamma, mu, Pr
        p.cfl_c, p.cfl_v, p.Cs = cfl_c, cfl_v, Cs
        p.limiter, p.max_halvings, p.precision, p.rk = limiter, max_halvings, precision, rk
        self.grid = grid
        self.params = p
        h = C.c_void_p()
        _check(lib().af_init_grid(C.byref(p), C.byref(h)))
        self.ctx = h
        nsides = 2 if grid.dim == 1 else 4
        for side in range(nsides):
            _check(lib().af_set_bc(self.ctx, side, int(grid.bc[side])))
        if bcstate is not None:  # 1D Dirichlet states [x-low, x-high]
            for side in range(2):
                arr = (C.c_double * 3)(*[float(v) for v in bcstate[side]])
                _check(lib().af_set_bc_state(self.ctx, side, arr))
        self.state_len = int(lib().af_state_len(self.ctx))
        self.ws_bytes = int(lib().af_workspace_bytes(self.ctx))
        if self.state_len != grid.state_len:
            raise AFError(AF_E_ARG, "state length mismatch between library and grid")
        self.device = torch.device(device)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.dt_dev = torch.zeros(1, dtype=torch.float64, device=self.device)
        _check(lib().af_reset_flags(self.ctx, _ptr(self.ws), _stream(None)))

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                lib().af_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # -- marshalling of the C ABI ------------------------------------------
    def to_device(self, U) -> torch.Tensor:
        return torch.as_tensor(U, dtype=torch.float64).to(self.device).contiguous()

    def af_rk_stage(self, k: int, Un, Uk, Uout, dt: float | None = None, dt_dev=None, stream=None):
        _check(lib().af_rk_stage(self.ctx, k, _ptr(dt_dev), 0.0 if dt is None else float(dt),
                                 _ptr(Un), _ptr(Uk), _ptr(Uout), _ptr(self.ws), _stream(stream)))

    def af_cfl_dt(self, U, t: float = 0.0, t_final: float = 1e300, dt_dev=None, stream=None):
        out = self.dt_dev if dt_dev is None else dt_dev
        _check(lib().af_cfl_dt(self.ctx, _ptr(U), t, t_final, _ptr(out), _ptr(self.ws),
                               _stream(stream)))
        return out

    def af_step(self, U, dt: float = 0.0, t: float = 0.0, t_final: float = 1e300, stream=None):
        """returns (status, dt_used, halvings); raises only on argument/HIP errors"""
        dtu = C.c_double()
        h = C.c_int()
        st = lib().af_step(self.ctx, _ptr(U), _ptr(self.ws), _stream(stream), dt, t, t_final,
                           C.byref(dtu), C.byref(h))
        if st in (AF_E_ARG, AF_E_HIP):
            _check(st)
        return st, dtu.value, h.value

    def af_step_noalloc(self, U, dt: float = 0.0, t: float = 0.0, t_final: float = 1e300,
                        stream=None):
        """af_step on the library's own scratch array instead of this
        solver's workspace; returns (status, dt_used, halvings)"""
        dtu = C.c_double()
        h = C.c_int()
        st = lib().af_step_noalloc(self.ctx, _ptr(U), _stream(stream), dt, t, t_final,
                                   C.byref(dtu), C.byref(h))
        if st in (AF_E_ARG, AF_E_HIP):
            _check(st)
        return st, dtu.value, h.value

    def af_run(self, U, t0: float, t_final: float, max_steps: int, check_every: int = 50,
               stream=None):
        ns = C.c_long()
        t = C.c_double()
        st = lib().af_run(self.ctx, _ptr(U), _ptr(self.ws), _stream(stream), t0, t_final,
                          max_steps, check_every, C.byref(ns), C.byref(t))
        if st in (AF_E_ARG, AF_E_HIP):
            _check(st)
        return st, ns.value, t.value

    def af_run_graph(self, U, t0: float, t_final: float, max_steps: int,
                     attempts_per_slot: int = 4, stream=None):
        """af_run with the step decisions on the device and graph replay;
        returns (status, steps, t, attempts)"""
        ns = C.c_long()
        t = C.c_double()
        att = C.c_long()
        st = lib().af_run_graph(self.ctx, _ptr(U), _ptr(self.ws), _stream(stream), t0, t_final,
                                max_steps, attempts_per_slot, C.byref(ns), C.byref(t),
                                C.byref(att))
        if st in (AF_E_ARG, AF_E_HIP):
            _check(st)
        return st, ns.value, t.value, att.value

    def af_read_flags(self, stream=None) -> int:
        f = C.c_int()
        _check(lib().af_read_flags(self.ctx, _ptr(self.ws), C.byref(f), _stream(stream)))
        return f.value

    def af_reset_flags(self, stream=None):
        _check(lib().af_reset_flags(self.ctx, _ptr(self.ws), _stream(stream)))

    def af_set_state(self, U_dev, U_host, stream=None):
        """copy a host state (numpy float64, af_state_len values) to a device state"""
        import numpy as np
        h = np.ascontiguousarray(U_host, dtype=np.float64)
        if h.size != self.state_len:
            raise ValueError(f"host state has {h.size} values, expected {self.state_len}")
        _check(lib().af_set_state(self.ctx, _ptr(U_dev), h.ctypes.data_as(C.c_void_p),
                                  _stream(stream)))

    def af_get_state(self, U_dev, stream=None):
        """copy a device state to a new host array"""
        import numpy as np
        h = np.empty(self.state_len, dtype=np.float64)
        _check(lib().af_get_state(self.ctx, _ptr(U_dev), h.ctypes.data_as(C.c_void_p),
                                  _stream(stream)))
        return h

    def af_check_admissible(self, U, stream=None) -> int:
        """number of DOF sites of U with non-positive density or pressure"""
        n = C.c_long()
        _check(lib().af_check_admissible(self.ctx, _ptr(U), _ptr(self.ws), _stream(stream),
                                         C.byref(n)))
        return n.value

    def af_step_source(self, U, dt: float, sources: list, stream=None):
        """one step with source states (device tensors) at the stage times;
        returns the status"""
        arr = (C.c_void_p * len(sources))(*[S.data_ptr() for S in sources])
        st = lib().af_step_source(self.ctx, _ptr(U), _ptr(self.ws), _stream(stream), dt, arr,
                                  len(sources))
        if st in (AF_E_ARG, AF_E_HIP):
            _check(st)
        return st

    # -- the learned blend (2D) --------------------------------------------
    @property
    def face_count(self) -> int:
        return int(lib().af_face_count(self.ctx))

    def af_blend_features(self, U, stream=None) -> torch.Tensor:
        """(faces, 40) float32 features of the device state U"""
        out = torch.empty((self.face_count, 40), dtype=torch.float32, device=self.device)
        _check(lib().af_blend_features(self.ctx, _ptr(U), _ptr(out), _stream(stream)))
        return out

    def af_set_blend_net(self, params):
        """the network (af_mlp_param_count float32 values on the device); the
        solver keeps a reference to it"""
        if params is not None:
            params = params.contiguous()
            if params.dtype != torch.float32 or params.numel() != mlp_param_count():
                raise ValueError("params: float32 tensor of af_mlp_param_count values")
        self.net = params
        _check(lib().af_set_blend_net(self.ctx, _ptr(params)))

    def af_blend_infer(self, U, stream=None) -> torch.Tensor:
        out = torch.empty(self.face_count, dtype=torch.float32, device=self.device)
        _check(lib().af_blend_infer(self.ctx, _ptr(U), _ptr(out), _ptr(self.ws), _stream(stream)))
        return out

    def af_rk_stage_blend(self, k: int, Un, Uk, Uout, dt: float | None = None, dt_dev=None,
                          theta=None, theta_s_out=None, stream=None):
        _check(lib().af_rk_stage_blend(self.ctx, k, _ptr(dt_dev), 0.0 if dt is None else float(dt),
                                       _ptr(Un), _ptr(Uk), _ptr(Uout), _ptr(theta),
                                       _ptr(theta_s_out), _ptr(self.ws), _stream(stream)))

    def af_timing(self, enable: bool):
        _check(lib().af_timing(self.ctx, 1 if enable else 0))

    def af_timing_read(self) -> dict:
        """{kind name: (launches, total ms)} since the previous read"""
        n = (C.c_long * K_COUNT)()
        ms = (C.c_double * K_COUNT)()
        _check(lib().af_timing_read(self.ctx, n, ms))
        return {KERNEL_KINDS.get(k, f"k{k}"): (n[k], ms[k]) for k in range(K_COUNT) if n[k]}


def stage_times(rk: int) -> list:
    c = (C.c_double * 5)()
    n = lib().af_stage_times(rk, c)
    if n < 0:
        raise ValueError("rk must be 3 or 54")
    return list(c)[:n]


def mlp_param_count() -> int:
    return int(lib().af_mlp_param_count())


def _grad_ws(n: int, device) -> torch.Tensor:
    nb = int(lib().af_mlp_grad_workspace_bytes(n))
    return torch.empty(nb, dtype=torch.uint8, device=device)


def mlp_grad(X, y, params, stream=None):
    """(gradient, loss) of the mean squared error of the network on rows X
    (n x 40 float32) against y (n), all on the device"""
    n = X.shape[0]
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    gws = _grad_ws(n, params.device)
    _check(lib().af_mlp_grad(_ptr(X), _ptr(y), n, _ptr(params), _ptr(grad), _ptr(loss), _ptr(gws),
                             _stream(stream)))
    return grad, loss


def mlp_adam(params, grad, m, v, step: int, lr: float, stream=None):
    _check(lib().af_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr,
                             _stream(stream)))


def mlp_train(X, y, params, m, v, step0: int, steps: int, batch: int, lr: float, stream=None):
    """`steps` Adam steps over minibatches of X, y in order; returns the last
    minibatch's loss (a device tensor)"""
    n = X.shape[0]
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    gws = _grad_ws(min(n, batch), params.device)
    _check(lib().af_mlp_train(_ptr(X), _ptr(y), n, _ptr(params), _ptr(grad), _ptr(m), _ptr(v),
                              step0, steps, batch, lr, _ptr(loss), _ptr(gws), _stream(stream)))
    return loss


def stage_variants() -> list:
    """the compiled 2D stage variants: (name, precision, tile height) each"""
    out = []
    for i in range(lib().af_stage_variant_count()):
        name, prec, ty = C.c_char_p(), C.c_int(), C.c_int()
        _check(lib().af_stage_variant_info(i, C.byref(name), C.byref(prec), C.byref(ty)))
        out.append((name.value.decode(), prec.value, ty.value))
    return out


class Batch:
    """A batch of 2D solvers (one precision) advanced together by af_batch_run:
    each stage of every instance is one persistent launch, each instance with
    its own time step and halving.  The solvers must outlive the batch."""

    def __init__(self, solvers: list):
        self.solvers = list(solvers)
        n = len(self.solvers)
        arr = (C.c_void_p * n)(*[s.ctx.value for s in self.solvers])
        h = C.c_void_p()
        _check(lib().af_batch_create(arr, n, C.byref(h)))
        self.h = h
        dev = self.solvers[0].device
        nb = int(lib().af_batch_workspace_bytes(h))
        self.ws = torch.empty(nb // 8 + 1, dtype=torch.float64, device=dev)

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and _lib is not None:
                _lib.af_batch_destroy(self.h)
        except Exception:
            pass

    def af_batch_run(self, states: list, t0: float, t_final: float, max_steps: int,
                     attempts_per_slot: int = 4, use_graph: bool = False, stream=None):
        """advance the device states in place; returns per-instance
        (status, steps, t, attempts) lists"""
        n = len(self.solvers)
        if len(states) != n:
            raise ValueError("one state per instance")
        ptrs = (C.c_void_p * n)(*[U.data_ptr() for U in states])
        steps = (C.c_long * n)()
        t = (C.c_double * n)()
        st = (C.c_int * n)()
        att = (C.c_long * n)()
        _check(lib().af_batch_run(self.h, ptrs, _ptr(self.ws), _stream(stream), t0, t_final,
                                  max_steps, attempts_per_slot, 1 if use_graph else 0, steps, t,
                                  st, att))
        return list(st), list(steps), list(t), list(att)

    @property
    def variant(self) -> int:
        """index (into stage_variants()) of the stage variant the batch uses"""
        return int(lib().af_batch_variant(self.h))

    @variant.setter
    def variant(self, i: int):
        _check(lib().af_batch_set_variant(self.h, int(i)))

    def af_batch_tune(self, states: list, t0: float, t_final: float, reps: int = 3,
                      stream=None) -> list:
        """time every stage variant of the batch's precision on one step slot
        from the given states and keep the fastest; returns the time per slot
        of each variant in microseconds (-1 for the other precision)"""
        n = len(self.solvers)
        if len(states) != n:
            raise ValueError("one state per instance")
        ptrs = (C.c_void_p * n)(*[U.data_ptr() for U in states])
        nv = lib().af_stage_variant_count()
        us = (C.c_double * nv)()
        _check(lib().af_batch_tune(self.h, ptrs, _ptr(self.ws), _stream(stream), t0, t_final,
                                   reps, us))
        return list(us)
