"""Pins of the oracle's semi-discrete right-hand side against the exact
Navier-Stokes right-hand side (sympy, written from the PDE in conservative
form with the Newtonian stress and Fourier heat flux, Sec. 1), and of the
whole scheme against the exact Euler density wave.

Accuracy statements used (all follow from the paper's operators):
* cubic conservative fields make the Simpson centre reconstruction exact
  (1D Sec. 2.1, 2D Sec. 2.2, exact for bicubics), so the point residual and
  the cell-average residual then converge at fourth order for both the
  inviscid (the D+/D- dissipation is a fourth difference, zero on cubics) and
  the viscous parts;
* for general smooth periodic data the Simpson centres carry an O(dx^4) error
  that the symmetric D^2 stencil divides by dx^2: the viscous point residual
  is then second order where a D^2 line passes through centres (1D points, 2D
  edge points) and fourth order where none does (2D corners); the inviscid
  point residual is third order, and the 1D cell-average inviscid residual is
  exact (point values are exact);
* the full scheme (SSP-RK3 with dt ~ dx^(4/3)) converges at fourth order to
  the exact Euler solution rho(x - t), u = 1, p = 1 at mu = 0 (Sec. 4 claims
  fourth order; mu = 0 reduces the method to inviscid AF).
A dropped term, a wrong sign, a wrong index or a transposed operand in the
residual shows up here as an O(1) error or an order drop.
"""
import numpy as np
import pytest
import sympy as sp

import oracle as O
from exact_ns import cell_avg_1d, cell_avg_2d, ev, rhs_1d, rhs_2d, x, y
from paper_2609_29081_amd import workloads as W

GAMMA, PR, MU = 1.4, 0.72, 0.05


def orders(errs):
    return [np.log2(a / b) for a, b in zip(errs[:-1], errs[1:])]


def lam1(exprs):
    f = sp.lambdify(x, exprs, "numpy")
    return lambda xx: tuple(np.broadcast_to(np.asarray(a, float), np.shape(xx)) for a in f(xx))


def lam2(exprs):
    f = sp.lambdify((x, y), exprs, "numpy")
    return lambda xx, yy: tuple(np.broadcast_to(np.asarray(a, float), np.shape(xx)) for a in f(xx, yy))


def residual_errors_1d(prim, Ns, bc, margin):
    rho, u, p = prim
    inv, vis = rhs_1d(rho, u, p, GAMMA, MU, PR)
    f = lam1(prim)
    out = []
    for N in Ns:
        g = W.Grid(dim=1, n1=N, bc=(bc,) * 4)
        U = W.make_state(g, f, GAMMA)
        P0 = g.split(O.rhs(O.make_cfg(g, mu=0.0, Pr=PR, limiter=0), U))
        P1 = g.split(O.rhs(O.make_cfg(g, mu=MU, Pr=PR, limiter=0), U))
        xs, _ = g.point_coords("pts")
        sp_ = slice(margin, g.n1x - margin)
        sc = slice(margin, N - margin)
        e = [max(np.abs(P0["pts"][k, 0] - ev(inv[k], xs))[sp_].max() for k in range(3)),
             max(np.abs(P1["pts"][k, 0] - P0["pts"][k, 0] - ev(vis[k], xs))[sp_].max() for k in range(3)),
             max(np.abs(P0["avg"][k, 0] - cell_avg_1d(inv[k], g))[sc].max() for k in range(3)),
             max(np.abs(P1["avg"][k, 0] - P0["avg"][k, 0] - cell_avg_1d(vis[k], g))[sc].max() for k in range(3))]
        out.append(e)
    return np.array(out)


def test_residual_1d_cubic_fields_fourth_order():
    R = 1 + 0.3 * x - 0.2 * x ** 2 + 0.25 * x ** 3
    M = 0.4 - 0.5 * x + 0.3 * x ** 2 + 0.2 * x ** 3
    E = 3 + 0.4 * x + 0.5 * x ** 2 - 0.6 * x ** 3
    prim = (R, M / R, (GAMMA - 1) * (E - M ** 2 / (2 * R)))
    e = residual_errors_1d(prim, (16, 32, 64, 128), W.OUTFLOW, 4)
    o_pi, o_pv, o_cv = orders(e[:, 0]), orders(e[:, 1]), orders(e[:, 3])
    assert o_pi[-1] > 3.5, o_pi
    assert o_pv[-1] > 3.5, o_pv
    assert o_cv[-1] > 3.5, o_cv
    assert e[:, 2].max() < 1e-11       # inviscid cell residual exact up to rounding
    assert e[-1, 1] < 1e-9


def test_residual_1d_periodic_trig_orders():
    prim = (1 + 0.2 * sp.sin(2 * sp.pi * x), 0.5 + 0.1 * sp.cos(2 * sp.pi * x),
            1 + 0.1 * sp.sin(4 * sp.pi * x + 0.3))
    e = residual_errors_1d(prim, (32, 64, 128, 256), W.PERIODIC, 0)
    o_pi, o_pv, o_cv = orders(e[:, 0]), orders(e[:, 1]), orders(e[:, 3])
    assert 2.8 < o_pi[-1] < 3.3, o_pi
    assert 1.8 < o_pv[-1] < 2.3, o_pv      # Simpson-centre error / dx^2
    assert o_cv[-1] > 3.7, o_cv
    assert e[:, 2].max() < 1e-11


def test_residual_2d_bicubic_fields_fourth_order():
    R = (1 + 0.2 * x - 0.1 * x ** 2 + 0.1 * x ** 3) * (1 + 0.1 * y + 0.2 * y ** 2 - 0.1 * y ** 3)
    MX = 0.3 + 0.2 * x - 0.3 * x * y + 0.1 * x ** 3 * y ** 2 - 0.2 * y ** 3
    MY = -0.2 + 0.1 * y + 0.2 * x * y - 0.15 * x ** 2 * y ** 3 + 0.1 * x ** 3
    E = 3 + 0.2 * x - 0.1 * y + 0.3 * x ** 2 * y - 0.2 * x ** 3 + 0.1 * y ** 3 * x
    prim = (R, MX / R, MY / R, (GAMMA - 1) * (E - (MX ** 2 + MY ** 2) / (2 * R)))
    inv, vis = rhs_2d(*prim, GAMMA, MU, PR)
    f = lam2(prim)
    errs = []
    for N in (16, 32, 64):
        g = W.Grid(dim=2, n1=N, n2=N, bc=(W.OUTFLOW,) * 4)
        U = W.make_state(g, f, GAMMA)
        P0 = g.split(O.rhs(O.make_cfg(g, mu=0.0, Pr=PR, limiter=0), U))
        P1 = g.split(O.rhs(O.make_cfg(g, mu=MU, Pr=PR, limiter=0), U))
        s = (slice(4, -4), slice(4, -4))
        row = []
        for name in ("xe", "ye", "co"):
            X, Y = g.point_coords(name)
            row.append(max(np.abs(P0[name][k] - ev(inv[k], X, Y))[s].max() for k in range(4)))
            row.append(max(np.abs(P1[name][k] - P0[name][k] - ev(vis[k], X, Y))[s].max() for k in range(4)))
        row.append(max(np.abs(P0["avg"][k] - cell_avg_2d(inv[k], g))[s].max() for k in range(4)))
        row.append(max(np.abs(P1["avg"][k] - P0["avg"][k] - cell_avg_2d(vis[k], g))[s].max() for k in range(4)))
        errs.append(row)
    errs = np.array(errs)
    for col in range(errs.shape[1]):
        o = orders(errs[:, col])
        assert o[-1] > 3.5, (col, o, errs[:, col])


def test_residual_2d_periodic_smooth_orders():
    """general smooth data: inviscid points third order; the viscous residual
    is second order at edge points, whose D^2 lines pass through Simpson
    centres (an O(dx^4) error summed by a symmetric stencil and divided by
    dx^2), and fourth order at corners, whose D^2 lines hold no centre (the
    antisymmetric D_c of the mixed terms only differences the smooth centre
    error); cell averages are fourth order"""
    prim = (1 + 0.2 * sp.sin(2 * sp.pi * (x + y)), 0.6 + 0.1 * sp.cos(2 * sp.pi * x) * sp.sin(2 * sp.pi * y),
            -0.4 + 0.1 * sp.sin(2 * sp.pi * (x - 2 * y)), 1 + 0.1 * sp.cos(2 * sp.pi * (2 * x + y)))
    inv, vis = rhs_2d(*prim, GAMMA, MU, PR)
    f = lam2(prim)
    errs = []
    for N in (32, 64, 128):
        g = W.Grid(dim=2, n1=N, n2=N)
        U = W.make_state(g, f, GAMMA)
        P0 = g.split(O.rhs(O.make_cfg(g, mu=0.0, Pr=PR, limiter=0), U))
        P1 = g.split(O.rhs(O.make_cfg(g, mu=MU, Pr=PR, limiter=0), U))
        row = []
        for name in ("co", "xe", "ye"):
            X, Y = g.point_coords(name)
            row.append(max(np.abs(P0[name][k] - ev(inv[k], X, Y)).max() for k in range(4)))
            row.append(max(np.abs(P1[name][k] - P0[name][k] - ev(vis[k], X, Y)).max() for k in range(4)))
        row.append(max(np.abs(P0["avg"][k] - cell_avg_2d(inv[k], g)).max() for k in range(4)))
        row.append(max(np.abs(P1["avg"][k] - P0["avg"][k] - cell_avg_2d(vis[k], g)).max() for k in range(4)))
        errs.append(row)
    errs = np.array(errs)
    o = [orders(errs[:, c])[-1] for c in range(errs.shape[1])]
    assert 2.7 < o[0] < 3.4, o      # co inviscid
    assert o[1] > 3.6, o            # co viscous
    assert 2.7 < o[2] < 3.4, o      # xe inviscid
    assert 1.7 < o[3] < 2.4, o      # xe viscous
    assert 2.7 < o[4] < 3.4, o      # ye inviscid
    assert 1.7 < o[5] < 2.4, o      # ye viscous
    assert o[6] > 3.6, o            # cells inviscid
    assert o[7] > 3.6, o            # cells viscous


@pytest.mark.parametrize("limiter", [0, O.LIM_ALL])
def test_euler_density_wave_fourth_order(limiter):
    """mu = 0: the method is inviscid AF; rho(x-t) is an exact solution"""
    errs = []
    T = 0.5
    for N in (16, 32, 64, 128):
        g, f = W.density_wave_1d(N)
        U = W.make_state(g, f, GAMMA)
        c = O.make_cfg(g, mu=0.0, limiter=limiter)
        nst = int(np.ceil(T / (0.5 * g.dx ** (4.0 / 3.0) / 2.4)))
        dt = T / nst
        for _ in range(nst):
            st, _, h, _ = O.step(c, U, dt)
            assert st == 0 and h == 0
        Ue = W.make_state(g, lambda xx: f(xx - T), GAMMA)
        P, Pe = g.split(U), g.split(Ue)
        errs.append([np.abs(P["avg"][0] - Pe["avg"][0]).mean(), np.abs(P["pts"][0] - Pe["pts"][0]).mean()])
    errs = np.array(errs)
    for col in range(2):
        o = orders(errs[:, col])
        assert min(o) > 3.8, o
