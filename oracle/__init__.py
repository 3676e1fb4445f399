"""ctypes binding of the FP64 CPU oracle (oracle/af_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "af_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

LIM_SMOOTH, LIM_PP, LIM_POINT, LIM_CENTRE, LIM_LOWONLY = 1, 2, 4, 8, 16
DIRICHLET = 4
LIM_ALL = LIM_SMOOTH | LIM_PP | LIM_POINT | LIM_CENTRE
LIM_PEXACT = 64   # theta^p as the root of the pressure quadratic (reading R-pquad)
FLAG_CELL_LOW, FLAG_POINT_LOW, FLAG_NONFINITE = 1, 2, 4


def build(force: bool = True) -> str:
    """compile the oracle with gcc (FP64, no contraction, OpenMP over rows)"""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
               "-o", LIB, SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return LIB


class Cfg(C.Structure):
    _fields_ = [("dim", C.c_int), ("n1", C.c_int), ("n2", C.c_int),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("gamma", C.c_double), ("mu", C.c_double), ("Pr", C.c_double),
                ("Cs", C.c_double), ("cfl_c", C.c_double), ("cfl_v", C.c_double),
                ("limiter", C.c_int), ("bc", C.c_int * 4), ("max_halvings", C.c_int),
                ("rk", C.c_int), ("bcstate", (C.c_double * 3) * 2)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        cp = C.POINTER(Cfg)
        L.orc_state_len.argtypes = [cp]
        L.orc_state_len.restype = C.c_long
        L.orc_fe.argtypes = [cp, dp, C.c_double, dp, dp, dp]
        L.orc_fe.restype = C.c_int
        L.orc_fe_blend.argtypes = [cp, dp, C.c_double, dp, dp, dp, dp]
        L.orc_fe_blend.restype = C.c_int
        L.orc_nfaces.argtypes = [cp]
        L.orc_nfaces.restype = C.c_long
        L.orc_blend_features.argtypes = [cp, dp, dp]
        L.orc_blend_features.restype = C.c_int
        L.orc_rhs.argtypes = [cp, dp, dp]
        L.orc_rhs.restype = None
        L.orc_dt.argtypes = [cp, dp]
        L.orc_dt.restype = C.c_double
        L.orc_dt_pp.argtypes = [cp, dp]
        L.orc_dt_pp.restype = C.c_double
        L.orc_step.argtypes = [cp, dp, C.c_double, C.c_double, C.c_double, dp,
                               C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_step.restype = C.c_int
        L.orc_run.argtypes = [cp, dp, C.c_double, C.c_double, C.c_long,
                              C.POINTER(C.c_long), dp]
        L.orc_run.restype = C.c_int
        L.orc_Theta.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_Theta.restype = C.c_double
        L.orc_theta_p_root.argtypes = [cp, dp, dp, C.c_double]
        L.orc_theta_p_root.restype = C.c_double
        L.orc_pressure.argtypes = [cp, dp]
        L.orc_pressure.restype = C.c_double
        L.orc_flux_c.argtypes = [cp, C.c_int, dp, dp]
        L.orc_flux_v.argtypes = [cp, C.c_int, dp, dp, dp]
        L.orc_bvisc.argtypes = [cp, C.c_int, dp, dp]
        L.orc_bvisc.restype = C.c_double
        for f in ("orc_op_dplus", "orc_op_dminus", "orc_op_dc"):
            getattr(L, f).argtypes = [dp, C.c_double]
            getattr(L, f).restype = C.c_double
        L.orc_op_d2.argtypes = [dp, dp, C.c_double]
        L.orc_op_d2.restype = C.c_double
        L.orc_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_cfg(grid, gamma=1.4, mu=1e-3, Pr=0.72, limiter=LIM_ALL, cfl_c=0.2, cfl_v=0.05,
             Cs=1.0, max_halvings=40, rk=3, bcstate=None) -> Cfg:
    c = Cfg()
    c.dim, c.n1, c.n2 = grid.dim, grid.n1, grid.n2
    c.x0, c.x1, c.y0, c.y1 = grid.x0, grid.x1, grid.y0, grid.y1
    c.gamma, c.mu, c.Pr, c.Cs = gamma, mu, Pr, Cs
    c.cfl_c, c.cfl_v = cfl_c, cfl_v
    c.limiter = limiter
    for k in range(4):
        c.bc[k] = int(grid.bc[k])
    c.max_halvings = max_halvings
    c.rk = rk
    if bcstate is not None:
        for side in range(2):
            for k in range(3):
                c.bcstate[side][k] = float(bcstate[side][k])
    return c


def nfaces(cfg: Cfg) -> int:
    if cfg.dim == 1:
        return cfg.n1 + 1
    return cfg.n2 * (cfg.n1 + 1) + (cfg.n2 + 1) * cfg.n1


def fe(cfg: Cfg, U: np.ndarray, dt: float, want_theta: bool = False):
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.empty_like(U)
    if want_theta:
        ts = np.empty(nfaces(cfg))
        tp = np.empty(nfaces(cfg))
        fl = lib().orc_fe(C.byref(cfg), _p(U), dt, _p(out), _p(ts), _p(tp))
        return out, fl, ts, tp
    fl = lib().orc_fe(C.byref(cfg), _p(U), dt, _p(out), None, None)
    return out, fl


def fe_blend(cfg: Cfg, U: np.ndarray, dt: float, theta_nn: np.ndarray, want_theta: bool = False):
    """2D forward-Euler stage with a given blend coefficient per face in
    place of theta^s (F = F^L + theta_nn theta^rho theta^p (F^H - F^L));
    returns (Ufe, flags) or, with want_theta, also the coefficient used in
    theta^s's place and theta^rho theta^p per face"""
    U = np.ascontiguousarray(U, dtype=np.float64)
    th = np.ascontiguousarray(theta_nn, dtype=np.float64)
    assert th.shape == (nfaces(cfg),)
    out = np.empty_like(U)
    ts = np.empty(nfaces(cfg)) if want_theta else None
    tp = np.empty(nfaces(cfg)) if want_theta else None
    fl = lib().orc_fe_blend(C.byref(cfg), _p(U), dt, _p(th), _p(out),
                            _p(ts) if want_theta else None, _p(tp) if want_theta else None)
    if fl < 0:
        raise ValueError("fe_blend needs a 2D config")
    return (out, fl, ts, tp) if want_theta else (out, fl)


def blend_features(cfg: Cfg, U: np.ndarray) -> np.ndarray:
    """the 40 features of every face (2D), shape (nfaces, 40)"""
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.empty((nfaces(cfg), 40))
    if lib().orc_blend_features(C.byref(cfg), _p(U), _p(out)) < 0:
        raise ValueError("blend_features needs a 2D config")
    return out


# Shu-Osher coefficients of the two integrators, for steps with a source
# term (the C oracle's orc_step covers the source-free steps): SSP-RK3, and
# Spiteri and Ruuth's SSPRK(5,4), the five-stage fourth-order SSP method
# Sec. 2.3 names
_RK54_A = dict(a20=0.444370493651235, a21=0.555629506348765, a30=0.620101851488403,
               a32=0.379898148511597, a40=0.178079954393132, a43=0.821920045606868,
               a52=0.517231671970585, a53=0.096059710526147, a54=0.386708617503269)
_RK54_B = dict(b10=0.391752226571890, b21=0.368410593050371, b32=0.251891774271694,
               b43=0.544974750228521, b54=0.226007483236906)


def stage_times(rk: int) -> list:
    """times of the stage inputs as fractions of dt"""
    if rk == 3:
        return [0.0, 1.0, 0.5]
    A, B = _RK54_A, _RK54_B
    c1 = B["b10"]
    c2 = A["a21"] * c1 + B["b21"]
    c3 = A["a32"] * c2 + B["b32"]
    c4 = A["a43"] * c3 + B["b43"]
    return [0.0, c1, c2, c3, c4]


def step_source(cfg: Cfg, U: np.ndarray, dt: float, S: list):
    """one step of dU/dt = L(U) + S(t) with a given dt and no halving:
    every forward-Euler step is the limited FE of L followed by + tau S_k,
    S_k (state-shaped) being the source at the k-th stage input's time
    (stage_times).  Returns (new state, flags)."""
    def fe_s(V, tau, Sk):
        out, fl = fe(cfg, V, tau)
        return out + tau * Sk, fl
    if cfg.rk != 54:
        u1, f0 = fe_s(U, dt, S[0])
        e1, f1 = fe_s(u1, dt, S[1])
        u2 = 0.75 * U + 0.25 * e1
        e2, f2 = fe_s(u2, dt, S[2])
        return U / 3.0 + 2.0 / 3.0 * e2, f0 | f1 | f2
    A, B = _RK54_A, _RK54_B
    u1, f0 = fe_s(U, B["b10"] * dt, S[0])
    e1, f1 = fe_s(u1, B["b21"] / A["a21"] * dt, S[1])
    u2 = A["a20"] * U + A["a21"] * e1
    e2, f2 = fe_s(u2, B["b32"] / A["a32"] * dt, S[2])
    u3 = A["a30"] * U + A["a32"] * e2
    e3, f3 = fe_s(u3, B["b43"] / A["a43"] * dt, S[3])
    u4 = A["a40"] * U + A["a43"] * e3
    e4, f4 = fe_s(u4, B["b54"] / A["a54"] * dt, S[4])
    return A["a52"] * u2 + A["a53"] * e3 + A["a54"] * e4, f0 | f1 | f2 | f3 | f4


def rhs(cfg: Cfg, U: np.ndarray) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.empty_like(U)
    lib().orc_rhs(C.byref(cfg), _p(U), _p(out))
    return out


def dt(cfg: Cfg, U: np.ndarray) -> float:
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().orc_dt(C.byref(cfg), _p(U))


def dt_pp(cfg: Cfg, U: np.ndarray) -> float:
    """the positivity theorem's sufficient time step (end of Sec. 3.4): the
    LLF intermediate-state bound for the cell averages and for the low-order
    point scheme"""
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().orc_dt_pp(C.byref(cfg), _p(U))


def step(cfg: Cfg, U: np.ndarray, dt: float = 0.0, t: float = 0.0, t_final: float = 1e30):
    """one step in place (SSP-RK3, or SSP-RK54 when cfg.rk == 54); returns
    (status, dt_used, halvings, flags)"""
    assert U.dtype == np.float64 and U.flags.c_contiguous
    dtu = C.c_double()
    h = C.c_int()
    fl = C.c_int()
    st = lib().orc_step(C.byref(cfg), _p(U), dt, t, t_final, C.byref(dtu), C.byref(h), C.byref(fl))
    return st, dtu.value, h.value, fl.value


def run(cfg: Cfg, U: np.ndarray, t0: float, t_final: float, max_steps: int = 1 << 40):
    assert U.dtype == np.float64 and U.flags.c_contiguous
    ns = C.c_long()
    t = C.c_double()
    st = lib().orc_run(C.byref(cfg), _p(U), t0, t_final, max_steps, C.byref(ns), C.byref(t))
    return st, ns.value, t.value


def theta(zL, zH, eps):
    return lib().orc_Theta(zL, zH, eps)


def theta_p_root(cfg, UL, UT, eps):
    """theta^p of the exact rule from UL toward UT (reading R-pquad)"""
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UT = np.ascontiguousarray(UT, dtype=np.float64)
    return lib().orc_theta_p_root(C.byref(cfg), _p(UL), _p(UT), eps)


def pressure(cfg, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().orc_pressure(C.byref(cfg), _p(U))


def flux_c(cfg, d, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    F = np.zeros(4)
    lib().orc_flux_c(C.byref(cfg), d, _p(U), _p(F))
    return F[:len(U)]


def flux_v(cfg, d, U, S):
    U = np.ascontiguousarray(U, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    F = np.zeros(4)
    lib().orc_flux_v(C.byref(cfg), d, _p(U), _p(S), _p(F))
    return F[:len(U)]


def bvisc(cfg, d, U, S):
    U = np.ascontiguousarray(U, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    return lib().orc_bvisc(C.byref(cfg), d, _p(U), _p(S))


def op(name: str, z, dx: float) -> float:
    z = np.ascontiguousarray(z, dtype=np.float64)
    return getattr(lib(), "orc_op_" + name)(_p(z), dx)


def op_d2(k, z, dx: float) -> float:
    k = np.ascontiguousarray(k, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    return lib().orc_op_d2(_p(k), _p(z), dx)


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> None:
    """threads of the oracle's OpenMP loops from now on"""
    lib().orc_set_threads(int(n))
