"""Seeded synthetic inputs: grids, initial data and state packing.

This module builds the inputs that both the HIP library and the CPU oracle
are fed.  It holds none of the Active Flux arithmetic: it only evaluates
initial conditions (given as primitive variables rho, u, v, p), converts them
to conservative variables, averages them over cells with tensor Gauss-Legendre
quadrature and samples them at the point degrees of freedom.

State layout (shared contract, documented in include/af.h):
  1D: [avg: 3 x n][pts: 3 x np]                      np = n or n+1
  2D: [avg: 4 x n2 x n1][xe: 4 x n2 x n1x][ye: 4 x n2y x n1][co: 4 x n2y x n1x]
      n1x = n1 if x is periodic else n1+1 (n2y likewise), x fastest.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Sequence

import numpy as np

PERIODIC, OUTFLOW, NOSLIP, SYMMETRY, DIRICHLET = 0, 1, 2, 3, 4


@dataclass
class Grid:
    dim: int
    n1: int
    n2: int = 1
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    bc: Sequence[int] = field(default_factory=lambda: (PERIODIC,) * 4)

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.n1

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / self.n2

    @property
    def ncomp(self) -> int:
        return 3 if self.dim == 1 else 4

    @property
    def n1x(self) -> int:
        return self.n1 if self.bc[0] == PERIODIC else self.n1 + 1

    @property
    def n2y(self) -> int:
        return self.n2 if self.bc[2] == PERIODIC else self.n2 + 1

    def blocks(self):
        """(name, rows, cols) of each DOF array, in storage order."""
        if self.dim == 1:
            return [("avg", 1, self.n1), ("pts", 1, self.n1x)]
        return [("avg", self.n2, self.n1), ("xe", self.n2, self.n1x),
                ("ye", self.n2y, self.n1), ("co", self.n2y, self.n1x)]

    @property
    def state_len(self) -> int:
        return self.ncomp * sum(r * c for _, r, c in self.blocks())

    @property
    def dof_sites(self) -> int:
        """number of DOF sites (each a vector of ncomp conservative values)"""
        return sum(r * c for _, r, c in self.blocks())

    def split(self, U: np.ndarray) -> dict:
        """views of a state vector as {name: array[ncomp, rows, cols]}"""
        out, off = {}, 0
        for name, r, c in self.blocks():
            n = self.ncomp * r * c
            out[name] = U[off:off + n].reshape(self.ncomp, r, c)
            off += n
        return out

    def point_coords(self, name: str):
        """physical coordinates (x, y) of the sites of one point array"""
        if self.dim == 1:
            return self.x0 + np.arange(self.n1x) * self.dx, None
        if name == "xe":
            xs = self.x0 + np.arange(self.n1x) * self.dx
            ys = self.y0 + (np.arange(self.n2) + 0.5) * self.dy
        elif name == "ye":
            xs = self.x0 + (np.arange(self.n1) + 0.5) * self.dx
            ys = self.y0 + np.arange(self.n2y) * self.dy
        else:
            xs = self.x0 + np.arange(self.n1x) * self.dx
            ys = self.y0 + np.arange(self.n2y) * self.dy
        return np.meshgrid(xs, ys)


def conservative(prim: Sequence[np.ndarray], gamma: float) -> list:
    """(rho,u,p) or (rho,u,v,p) -> (rho, rho u, [rho v,] E)"""
    if len(prim) == 3:
        r, u, p = prim
        return [r, r * u, p / (gamma - 1.0) + 0.5 * r * u * u]
    r, u, v, p = prim
    return [r, r * u, r * v, p / (gamma - 1.0) + 0.5 * r * (u * u + v * v)]


def make_state(grid: Grid, prim_fn: Callable, gamma: float, nq: int = 5) -> np.ndarray:
    """Cell averages by nq-point tensor Gauss-Legendre quadrature of the
    conservative variables, point values sampled exactly."""
    gx, gw = np.polynomial.legendre.leggauss(nq)
    gx = 0.5 * (gx + 1.0)
    gw = 0.5 * gw
    U = np.zeros(grid.state_len)
    parts = grid.split(U)
    if grid.dim == 1:
        xl = grid.x0 + np.arange(grid.n1) * grid.dx
        acc = [np.zeros(grid.n1) for _ in range(3)]
        for q in range(nq):
            cons = conservative(prim_fn(xl + gx[q] * grid.dx), gamma)
            for k in range(3):
                acc[k] += gw[q] * cons[k]
        for k in range(3):
            parts["avg"][k, 0] = acc[k]
        xs, _ = grid.point_coords("pts")
        cons = conservative(prim_fn(xs), gamma)
        for k in range(3):
            parts["pts"][k, 0] = cons[k]
        return U
    xl = grid.x0 + np.arange(grid.n1) * grid.dx
    yl = grid.y0 + np.arange(grid.n2) * grid.dy
    XL, YL = np.meshgrid(xl, yl)
    acc = [np.zeros((grid.n2, grid.n1)) for _ in range(4)]
    for a in range(nq):
        for b in range(nq):
            cons = conservative(prim_fn(XL + gx[a] * grid.dx, YL + gx[b] * grid.dy), gamma)
            for k in range(4):
                acc[k] += gw[a] * gw[b] * cons[k]
    for k in range(4):
        parts["avg"][k] = acc[k]
    for name in ("xe", "ye", "co"):
        X, Y = grid.point_coords(name)
        cons = conservative(prim_fn(X, Y), gamma)
        for k in range(4):
            parts[name][k] = cons[k]
    return U


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

@dataclass
class Physics:
    gamma: float = 1.4
    mu: float = 1e-3
    Pr: float = 0.72


def density_wave_1d(n: int, amp: float = 0.2):
    """1D periodic [0,1]: rho = 1 + amp sin(2 pi x), u = 1, p = 1."""
    g = Grid(dim=1, n1=n, bc=(PERIODIC, PERIODIC, PERIODIC, PERIODIC))

    def f(x):
        return (1.0 + amp * np.sin(2 * np.pi * x), np.ones_like(x), np.ones_like(x))
    return g, f


def vortex_wave_2d(n: int, strength: float = 0.5, r0: float = 0.1):
    """2D periodic [0,1]^2: rho = 1 + 0.2 sin(2 pi (x+y)), (u,v) = (1,1) plus a
    Gaussian vortex centred at (1/2,1/2) summed over the 3x3 periodic images,
    p = 1."""
    g = Grid(dim=2, n1=n, n2=n)

    def f(x, y):
        du = np.zeros_like(x)
        dv = np.zeros_like(x)
        for sx in (-1.0, 0.0, 1.0):
            for sy in (-1.0, 0.0, 1.0):
                xx = x - 0.5 - sx
                yy = y - 0.5 - sy
                psi = np.exp(-(xx * xx + yy * yy) / (2 * r0 * r0))
                du += -strength * yy * psi / r0
                dv += strength * xx * psi / r0
        return (1.0 + 0.2 * np.sin(2 * np.pi * (x + y)), 1.0 + du, 1.0 + dv, np.ones_like(x))
    return g, f


def shock_tube_2d(n1: int = 1000, n2: int = 500, gamma: float = 1.4,
                  rho_left: float = 120.0, rho_right: float = 1.2):
    """Viscous shock tube on [0,1]x[0,0.5]: diaphragm at x=1/2 (a point on the
    line x=1/2 takes the right state), p = rho/gamma, at rest; no-slip
    adiabatic walls at x=0, x=1, y=0, symmetry at y=0.5."""
    g = Grid(dim=2, n1=n1, n2=n2, x0=0.0, x1=1.0, y0=0.0, y1=0.5,
             bc=(NOSLIP, NOSLIP, NOSLIP, SYMMETRY))

    def f(x, y):
        left = x < 0.5
        r = np.where(left, rho_left, rho_right)
        z = np.zeros_like(x)
        return (r, z, z.copy(), r / gamma)
    return g, f


def shock_tube_sweep(n: int = 64, seed: int = 0, gamma: float = 1.4,
                     n1_choices=tuple(range(128, 1025, 64))):
    """Parameter sweep of viscous shock tubes (the shock tube above with
    random parameters): for each of n instances, drawn in this order from
    numpy's default_rng(seed), Re ~ U[200, 1000] (mu = 1/Re), density ratio
    r ~ U[50, 200] (left rho = 1.2 r, p = rho/gamma; right rho = 1.2,
    p = 1.2/gamma) and N1 uniform on n1_choices with N2 = N1/2.  Returns a
    list of (grid, prim_fn, physics keywords) triples."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        re = float(rng.uniform(200.0, 1000.0))
        ratio = float(rng.uniform(50.0, 200.0))
        n1 = int(rng.choice(np.asarray(n1_choices)))
        g, f = shock_tube_2d(n1, n1 // 2, gamma=gamma, rho_left=1.2 * ratio, rho_right=1.2)
        out.append((g, f, dict(mu=1.0 / re, Pr=0.73, gamma=gamma)))
    return out


def mlp_init(seed: int = 0, nin: int = 40, nh: int = 64) -> np.ndarray:
    """Seeded initial parameters of the blend network (nin -> nh -> nh -> 1),
    as one float32 vector [W1 (nh x nin, row-major), b1, W2 (nh x nh), b2,
    w3 (nh), b3]: Glorot-uniform weights from numpy's default_rng(seed),
    zero hidden biases, output bias 1/2."""
    rng = np.random.default_rng(seed)

    def glorot(fan_out, fan_in):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, size=(fan_out, fan_in))
    parts = [glorot(nh, nin).ravel(), np.zeros(nh), glorot(nh, nh).ravel(), np.zeros(nh),
             glorot(1, nh).ravel(), np.array([0.5])]
    return np.concatenate(parts).astype(np.float32)


def balanced_rows(y: np.ndarray, seed: int = 0, ratio: float = 3.0, below: float = 0.999,
                  total: int = 0) -> np.ndarray:
    """Row indices of a training set for the blend network: every row whose
    target is below `below` (the faces where the smoothness blend acts, a
    few per cent of a shock-tube grid) and `ratio` times as many of the
    other rows -- or, with total > 0, as many of the others as make `total`
    rows in all (at least `ratio` times as many when there are enough) --
    drawn without replacement from default_rng(seed), in a shuffled order."""
    rng = np.random.default_rng(seed)
    y = np.asarray(y)
    lo = np.flatnonzero(y < below)
    hi = np.flatnonzero(~(y < below))
    k = int(ratio * max(len(lo), 1))
    if total > 0:
        k = max(k, total - len(lo))
    k = min(len(hi), k)
    idx = np.concatenate([lo, rng.choice(hi, size=k, replace=False)])
    return idx[rng.permutation(len(idx))]


def becker_shock_1d(n: int, M0: float = 3.0, mu: float = 1e-2, gamma: float = 1.4,
                    Pr: float = 0.75, u_inf: float = 0.2):
    """The moving viscous shock of the paper's 1D accuracy test (Sec. 4; the
    exact solution Becker derived for Pr = 3/4): domain [-1, 1.5], shock at
    x = u_inf t, rho_L = w_L = m_0 = 1, upstream Mach number M0 in the
    shock frame; Dirichlet sides.  w(xi) (velocity relative to the shock,
    xi = x - u_inf t) solves
      xi = 2 mu gamma / ((gamma+1) m0 Pr) * [wL/(wL-wR) ln((wL-w)/(wL-w0))
                                             - wR/(wL-wR) ln((w-wR)/(w0-wR))],
    w0 = sqrt(wL wR), wR/wL = ((gamma-1) + 2/M0^2)/(gamma+1); then
    rho = m0/w, u = u_inf + w, e = ((gamma+1)/(gamma-1) w0^2 - w^2)/(2 gamma),
    p = (gamma-1) rho e.  Returns (grid, prim(x, t), Dirichlet states
    [left, right] as conservative (rho, rho u, E))."""
    wL, m0 = 1.0, 1.0
    wR = wL * ((gamma - 1.0) + 2.0 / M0 ** 2) / (gamma + 1.0)
    w0 = np.sqrt(wL * wR)
    c = 2.0 * mu * gamma / ((gamma + 1.0) * m0 * Pr)

    def xi_of(w):
        with np.errstate(divide="ignore"):  # +-inf at the end states
            return c * (wL / (wL - wR) * np.log((wL - w) / (wL - w0))
                        - wR / (wL - wR) * np.log((w - wR) / (w0 - wR)))

    def w_of(xi):
        # xi(w) decreases from +inf (w -> wR) to -inf (w -> wL): bisection
        xi = np.asarray(xi, dtype=np.float64)
        lo = np.full(xi.shape, wR)
        hi = np.full(xi.shape, wL)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if np.all((mid == lo) | (mid == hi)):
                break
            big = xi_of(mid) > xi  # mid is too close to wR
            lo = np.where(big, mid, lo)
            hi = np.where(big, hi, mid)
        return 0.5 * (lo + hi)

    def prim(x, t=0.0):
        w = w_of(np.asarray(x) - u_inf * t)
        rho = m0 / w
        e = ((gamma + 1.0) / (gamma - 1.0) * w0 * w0 - w * w) / (2.0 * gamma)
        return (rho, u_inf + w, (gamma - 1.0) * rho * e)

    def cons(w):
        rho = m0 / w
        e = ((gamma + 1.0) / (gamma - 1.0) * w0 * w0 - w * w) / (2.0 * gamma)
        u = u_inf + w
        return [rho, rho * u, rho * e + 0.5 * rho * u * u]
    g = Grid(dim=1, n1=n, x0=-1.0, x1=1.5, bc=(DIRICHLET, DIRICHLET, DIRICHLET, DIRICHLET))
    return g, prim, [cons(wL), cons(wR)]


def taylor_green_2d(n: int, p0: float = 100.0, mu: float = 1e-5, gamma: float = 1.4,
                    Pr: float = 1.0):
    """The paper's manufactured Taylor-Green vortex (Sec. 4): periodic
    [0, 2 pi]^2, a(t) = exp(-2 mu t), b = cos 2x + cos 2y, rho = 1,
    (u, v) = a (sin x cos y, -cos x sin y), p = p0/(gamma-1) + a^2 b/4, with
    the energy source
      S_E = (p_t + u p_x + v p_y)/(gamma-1) - 4 mu a^2 cos^2 x cos^2 y
            - kappa lap p,
    p_t = -mu a^2 b, p_x = -a^2 sin(2x)/2, p_y = -a^2 sin(2y)/2,
    lap p = -a^2 b, kappa = gamma mu / ((gamma-1) Pr).  Returns (grid,
    prim(x, y, t), source(t)), source(t) being a state-shaped array of S
    (zero but for the energy component): cell averages by 5 x 5
    Gauss-Legendre quadrature, point values sampled."""
    two_pi = 2.0 * np.pi
    g = Grid(dim=2, n1=n, n2=n, x0=0.0, x1=two_pi, y0=0.0, y1=two_pi, bc=(PERIODIC,) * 4)
    kappa = gamma * mu / ((gamma - 1.0) * Pr)

    def prim(x, y, t=0.0):
        a = np.exp(-2.0 * mu * t)
        b = np.cos(2.0 * x) + np.cos(2.0 * y)
        return (np.ones_like(x), a * np.sin(x) * np.cos(y), -a * np.cos(x) * np.sin(y),
                p0 / (gamma - 1.0) + a * a * b / 4.0)

    def s_energy(x, y, t):
        a = np.exp(-2.0 * mu * t)
        b = np.cos(2.0 * x) + np.cos(2.0 * y)
        u, v = a * np.sin(x) * np.cos(y), -a * np.cos(x) * np.sin(y)
        pt, px, py = -mu * a * a * b, -a * a * np.sin(2.0 * x) / 2.0, -a * a * np.sin(2.0 * y) / 2.0
        lap = -a * a * b
        return ((pt + u * px + v * py) / (gamma - 1.0)
                - 4.0 * mu * a * a * np.cos(x) ** 2 * np.cos(y) ** 2 - kappa * lap)

    def source(t):
        S = np.zeros(g.state_len)
        parts = g.split(S)
        gx, gw = np.polynomial.legendre.leggauss(5)
        gx, gw = 0.5 * (gx + 1.0), 0.5 * gw
        xl = g.x0 + np.arange(g.n1) * g.dx
        yl = g.y0 + np.arange(g.n2) * g.dy
        XL, YL = np.meshgrid(xl, yl)
        acc = np.zeros((g.n2, g.n1))
        for qa in range(5):
            for qb in range(5):
                acc += gw[qa] * gw[qb] * s_energy(XL + gx[qa] * g.dx, YL + gx[qb] * g.dy, t)
        parts["avg"][3] = acc
        for name in ("xe", "ye", "co"):
            X, Y = g.point_coords(name)
            parts[name][3] = s_energy(X, Y, t)
        return S
    return g, prim, source


def leblanc_1d(n: int = 800):
    """LeBlanc-type near-vacuum Riemann problem on [-0.5,0.5], outflow."""
    g = Grid(dim=1, n1=n, x0=-0.5, x1=0.5, bc=(OUTFLOW, OUTFLOW, OUTFLOW, OUTFLOW))

    def f(x):
        left = x < -0.2
        r = np.where(left, 1.0, 1e-2)
        p = np.where(left, 6.666667e-2, 6.666667e-11)
        return (r, np.zeros_like(x), p)
    return g, f


def random_smooth_2d(n1: int, n2: int, seed: int, bc=(PERIODIC,) * 4,
                     x1: float = 1.0, y1: float = 1.0, amp: float = 0.1):
    """Seeded smooth periodic-in-[0,1] field made of a few random Fourier
    modes; admissible for amp <= 0.2."""
    rng = np.random.default_rng(seed)
    coef = rng.uniform(-1.0, 1.0, size=(4, 3, 4))
    g = Grid(dim=2, n1=n1, n2=n2, x1=x1, y1=y1, bc=tuple(bc))

    def field_(x, y, k):
        s = np.zeros_like(x)
        for m in range(3):
            a, b, c, d = coef[k, m]
            s += a * np.sin(2 * np.pi * ((m + 1) * x / x1 + b)) * np.cos(2 * np.pi * (m * y / y1 + c)) * (0.5 + 0.5 * d)
        return s

    def f(x, y):
        return (1.0 + amp * field_(x, y, 0), 0.5 + amp * field_(x, y, 1),
                -0.3 + amp * field_(x, y, 2), 1.0 + amp * field_(x, y, 3))
    return g, f


def double_rarefaction(n1: int, n2: int = 0, speed: float = 2.0, angle: float = 0.0):
    """Two rarefactions receding from x' = 1/2 (x' along direction `angle`),
    rho = 1, p = 0.4, |u| = speed: a near-vacuum centre that makes the
    density/pressure limiting act.  1D if n2 == 0, else a 2D grid on
    [0,1]^2 (periodic in y when angle == 0, outflow otherwise)."""
    if n2 == 0:
        g = Grid(dim=1, n1=n1, bc=(OUTFLOW,) * 4)

        def f(x):
            return (np.ones_like(x), np.where(x < 0.5, -speed, speed), 0.4 * np.ones_like(x))
        return g, f
    bc = (OUTFLOW, OUTFLOW, PERIODIC, PERIODIC) if angle == 0.0 else (OUTFLOW,) * 4
    g = Grid(dim=2, n1=n1, n2=n2, bc=bc)
    ca, sa = np.cos(angle), np.sin(angle)

    def f(x, y):
        s = np.where((x - 0.5) * ca + (y - 0.5) * sa < 0.0, -speed, speed)
        return (np.ones_like(x), s * ca, s * sa, 0.4 * np.ones_like(x))
    return g, f
