"""Pins of the oracle's viscous low-order point scheme (reading R-point of
the point-value limiting, Sec. 3.4) at mu > 0.

The scheme is the LLF scheme of eq. (ns_low_face_fluxes) on the half-spaced
lattice around each point: sites hold the point values and, at cell centres,
the cell averages; the gradient S of a site is the central difference of
Z = (0, u, v, T) over its two lattice neighbours in each direction (dx
apart); the link coefficient is lambda = max varrho_l + max b_l over the
link's two sites, b_l from the viscous splitting lemma (Sec. 3.1).

* On periodic data the oracle's low-order point values equal an independent,
  array-at-a-time evaluation of those formulas (stress and heat flux from the
  Newton/Fourier closure, b from the lemma's statement).
* The update is a convex combination of admissible states when
  dt <= min_l (dx_l/2) / (2 d max lambda_l) (the proposition on the LLF
  intermediate states, Sec. 3.1, on a lattice of spacing dx_l/2), so the
  low-order point values stay admissible and no point flag is raised on a
  cold state, rough at the lattice scale, where the viscous coefficient b
  dominates; four times that step does raise the flag, so the data test the
  bound.
"""
import numpy as np

import oracle as O
from paper_2609_29081_amd import workloads as W

GAMMA = 1.4


def half_lattice(g, U):
    """periodic state -> [4, 2 n2, 2 n1] half lattice (rows y, columns x):
    averages at centres, xe, ye and co at their sites"""
    P = g.split(U)
    H = np.empty((4, 2 * g.n2, 2 * g.n1))
    H[:, 1::2, 1::2] = P["avg"]
    H[:, 1::2, 0::2] = P["xe"]
    H[:, 0::2, 1::2] = P["ye"]
    H[:, 0::2, 0::2] = P["co"]
    return H


def llf_pieces(g, H, mu, Pr):
    """per site: the total fluxes F_x, F_y, |u_l| + c and b_l"""
    kap = GAMMA * mu / ((GAMMA - 1) * Pr)
    r = H[0]
    u, v = H[1] / r, H[2] / r
    p = (GAMMA - 1) * (H[3] - 0.5 * r * (u * u + v * v))
    T = p / r
    cs = np.sqrt(GAMMA * p / r)
    e = p / ((GAMMA - 1) * r)

    def ddx(z):  # neighbours half a cell away on either side: dx apart
        return (np.roll(z, -1, axis=1) - np.roll(z, 1, axis=1)) / g.dx

    def ddy(z):
        return (np.roll(z, -1, axis=0) - np.roll(z, 1, axis=0)) / g.dy

    ux, uy, vx, vy, Tx, Ty = ddx(u), ddy(u), ddx(v), ddy(v), ddx(T), ddy(T)
    txx = mu * (2 * ux - 2.0 / 3.0 * (ux + vy))
    tyy = mu * (2 * vy - 2.0 / 3.0 * (ux + vy))
    txy = mu * (uy + vx)
    qx, qy = -kap * Tx, -kap * Ty
    Fx = np.array([r * u, r * u * u + p, r * u * v, (H[3] + p) * u])
    Fy = np.array([r * v, r * u * v, r * v * v + p, (H[3] + p) * v])
    Fx -= np.array([0 * r, txx, txy, u * txx + v * txy - qx])
    Fy -= np.array([0 * r, txy, tyy, u * txy + v * tyy - qy])

    def b_of(q, t2):
        return (np.sqrt(r * r * q * q + 2 * r * r * e * t2) + r * np.abs(q)) / (2 * r * r * e)

    bx = b_of(qx, txx ** 2 + txy ** 2)
    by = b_of(qy, txy ** 2 + tyy ** 2)
    return Fx, Fy, np.abs(u) + cs, np.abs(v) + cs, bx, by


def link_lambda(a, b, axis):
    """lambda of the link between each site and its + neighbour along axis"""
    return np.maximum(a, np.roll(a, -1, axis=axis)) + np.maximum(b, np.roll(b, -1, axis=axis))


def low_order_points(g, H, dt, mu, Pr):
    Fx, Fy, ax, ay, bx, by = llf_pieces(g, H, mu, Pr)
    out = H.copy()
    for F, lam, h, axis in ((Fx, link_lambda(ax, bx, 1), g.dx, 2),
                            (Fy, link_lambda(ay, by, 0), g.dy, 1)):
        Fh = 0.5 * (F + np.roll(F, -1, axis=axis)) - 0.5 * lam * (np.roll(H, -1, axis=axis) - H)
        out -= 2.0 * dt / h * (Fh - np.roll(Fh, 1, axis=axis))
    return out


def sufficient_dt(g, H, mu, Pr):
    """min over l of (dx_l/2) / (2 d max lambda_l) over every lattice link"""
    _, _, ax, ay, bx, by = llf_pieces(g, H, mu, Pr)
    return min(0.5 * g.dx / (4 * link_lambda(ax, bx, 1).max()),
               0.5 * g.dy / (4 * link_lambda(ay, by, 0).max()))


def point_views(H):
    return {"xe": H[:, 1::2, 0::2], "ye": H[:, 0::2, 1::2], "co": H[:, 0::2, 0::2]}


def test_viscous_point_llf_matches_lattice_formulas():
    g, f = W.random_smooth_2d(12, 10, seed=21, amp=0.25, x1=1.2, y1=0.8)
    U = W.make_state(g, f, GAMMA)
    mu, Pr = 0.02, 0.72
    c = O.make_cfg(g, mu=mu, Pr=Pr, limiter=O.LIM_LOWONLY | O.LIM_POINT)
    H = half_lattice(g, U)
    dt = 0.5 * O.dt(c, U)
    out, fl = O.fe(c, U, dt)
    assert fl == 0
    ref = point_views(low_order_points(g, H, dt, mu, Pr))
    Q = g.split(out)
    for name in ("xe", "ye", "co"):
        for k in range(4):
            scale = np.abs(ref[name][k]).max() + np.abs(H[k]).max()
            assert np.abs(Q[name][k] - ref[name][k]).max() < 1e-13 * scale, (name, k)
    # the viscous part is not negligible on these data
    ref0 = point_views(low_order_points(g, H, dt, 0.0, Pr))
    assert max(np.abs(ref[n] - ref0[n]).max() for n in ref) > 1e-4


def rough_cold_state(seed=7, n1=16, n2=14, pmax=0.01):
    """every DOF an independent random state (seeded): density in [0.5, 2],
    velocity components in [-2, 2], pressure in [pmax/10, pmax] -- cold
    (internal energy below 1 % of the kinetic one) and rough at the lattice
    scale, so the viscous coefficient b exceeds |u| + c at many sites and the
    low-order update is near its positivity limit"""
    rng = np.random.default_rng(seed)
    g = W.Grid(dim=2, n1=n1, n2=n2)
    U = np.zeros(g.state_len)
    for arr in g.split(U).values():
        sh = arr[0].shape
        r = rng.uniform(0.5, 2.0, sh)
        u = rng.uniform(-2.0, 2.0, sh)
        v = rng.uniform(-2.0, 2.0, sh)
        p = rng.uniform(0.1 * pmax, pmax, sh)
        arr[:] = W.conservative([r, u, v, p], GAMMA)
    return g, U


def admissible_points(g, out):
    Q = g.split(out)
    ok = True
    for name in ("xe", "ye", "co"):
        r, mx, my, E = Q[name]
        p = (GAMMA - 1) * (E - 0.5 * (mx * mx + my * my) / r)
        ok = ok and r.min() > 0 and p.min() > 0
    return ok


def test_viscous_point_llf_admissible_under_its_sufficient_step():
    g, U = rough_cold_state()
    mu, Pr = 0.05, 0.72
    H = half_lattice(g, U)
    _, _, ax, ay, bx, by = llf_pieces(g, H, mu, Pr)
    assert (bx > ax).sum() > 200 and (by > ay).sum() > 200
    dt = sufficient_dt(g, H, mu, Pr)
    # centre values scaled toward the averages keep the (unused) high-order
    # residual finite on these rough data
    c = O.make_cfg(g, mu=mu, Pr=Pr, limiter=O.LIM_LOWONLY | O.LIM_POINT | O.LIM_CENTRE)
    out, fl = O.fe(c, U, dt)
    assert fl == 0
    assert admissible_points(g, out)
    # the bound is not vacuous on these data: four times the step fails
    out4, fl4 = O.fe(c, U, 4 * dt)
    assert fl4 & O.FLAG_POINT_LOW and not admissible_points(g, out4)
