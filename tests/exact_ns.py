"""Exact right-hand side of the compressible Navier-Stokes equations for
smooth primitive fields, by symbolic differentiation (sympy).

Written from the PDE itself (conservative form, Newtonian stress tensor and
Fourier heat flux, Sec. 1 of the paper), not from the diffusion-matrix form
the method uses, so it pins the discretisation independently.
"""
from __future__ import annotations

import numpy as np
import sympy as sp

x, y = sp.symbols("x y", real=True)


def rhs_1d(rho, u, p, gamma, mu, Pr):
    """returns numpy callables (avg-free) for dU/dt = -(F^c)_x + (F^v)_x,
    split into (inviscid, viscous) lists of 3 functions of x"""
    kap = gamma * mu / ((gamma - 1) * Pr)
    E = p / (gamma - 1) + rho * u ** 2 / 2
    Fc = [rho * u, rho * u ** 2 + p, (E + p) * u]
    T = p / rho
    tau = mu * (2 * sp.diff(u, x) - sp.Rational(2, 3) * sp.diff(u, x))
    q = -kap * sp.diff(T, x)
    Fv = [sp.Integer(0), tau, u * tau - q]
    inv = [sp.lambdify(x, -sp.diff(F, x), "numpy") for F in Fc]
    vis = [sp.lambdify(x, sp.diff(F, x), "numpy") for F in Fv]
    return inv, vis


def rhs_2d(rho, u, v, p, gamma, mu, Pr):
    kap = gamma * mu / ((gamma - 1) * Pr)
    E = p / (gamma - 1) + rho * (u ** 2 + v ** 2) / 2
    T = p / rho
    Fx = [rho * u, rho * u * u + p, rho * v * u, (E + p) * u]
    Fy = [rho * v, rho * u * v, rho * v * v + p, (E + p) * v]
    ux, uy, vx, vy = sp.diff(u, x), sp.diff(u, y), sp.diff(v, x), sp.diff(v, y)
    div = ux + vy
    txx = mu * (2 * ux - sp.Rational(2, 3) * div)
    tyy = mu * (2 * vy - sp.Rational(2, 3) * div)
    txy = mu * (uy + vx)
    qx = -kap * sp.diff(T, x)
    qy = -kap * sp.diff(T, y)
    Gx = [sp.Integer(0), txx, txy, u * txx + v * txy - qx]
    Gy = [sp.Integer(0), txy, tyy, u * txy + v * tyy - qy]
    inv = [sp.lambdify((x, y), -sp.diff(Fx[k], x) - sp.diff(Fy[k], y), "numpy") for k in range(4)]
    vis = [sp.lambdify((x, y), sp.diff(Gx[k], x) + sp.diff(Gy[k], y), "numpy") for k in range(4)]
    return inv, vis


def ev(fn, *args):
    """evaluate a lambdified function, broadcasting constants"""
    out = fn(*args)
    return np.broadcast_to(np.asarray(out, dtype=float), np.shape(args[0])).copy()


def cell_avg_1d(fn, grid, nq=6):
    gx, gw = np.polynomial.legendre.leggauss(nq)
    gx = 0.5 * (gx + 1)
    gw = 0.5 * gw
    xl = grid.x0 + np.arange(grid.n1) * grid.dx
    return sum(gw[q] * ev(fn, xl + gx[q] * grid.dx) for q in range(nq))


def cell_avg_2d(fn, grid, nq=6):
    gx, gw = np.polynomial.legendre.leggauss(nq)
    gx = 0.5 * (gx + 1)
    gw = 0.5 * gw
    xl = grid.x0 + np.arange(grid.n1) * grid.dx
    yl = grid.y0 + np.arange(grid.n2) * grid.dy
    XL, YL = np.meshgrid(xl, yl)
    acc = np.zeros_like(XL)
    for a in range(nq):
        for b in range(nq):
            acc += gw[a] * gw[b] * ev(fn, XL + gx[a] * grid.dx, YL + gx[b] * grid.dy)
    return acc
