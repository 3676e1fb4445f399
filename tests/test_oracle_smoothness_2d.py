"""Closed-form pins of the oracle's 2D smoothness blend theta^s (Sec. 3.2).

theta^s of a face is exp(-C_s phi_1 phi_2), each phi taken as the larger of
its values in the two cells beside the face, with
  phi_1 = max over both directions of |p+ - 2p + p-| / |p+ + 2p + p-|,
  phi_2 = max(-div u / sqrt(div u^2 + |curl u|^2 + 1e-13), 0),
from central differences of the cell averages' velocity and pressure.

The cell averages below are built so that every difference has a closed
form: velocities quadratic in the cell index (central differences of i^2
are exact: (i+1)^2 - (i-1)^2 = 4i) and pressures quadratic in each index
(second differences in closed form).  The expected theta^s is written from those
closed forms, not from the differences, so a dropped curl, a min in place of
a face max, phi_1 over one direction only or a lost regularisation changes
the result far beyond round-off.
"""
import numpy as np

import oracle as O
from paper_2609_29081_amd import workloads as W

GAMMA = 1.4


def state_from_cells(g, r, u, v, p):
    """state whose cell averages have the given primitive values per cell
    ([n2, n1] arrays) and whose point values are one admissible constant
    state (theta^s reads the averages only)"""
    U = np.zeros(g.state_len)
    P = g.split(U)
    E = p / (GAMMA - 1) + 0.5 * r * (u * u + v * v)
    for k, a in enumerate((r, r * u, r * v, E)):
        P["avg"][k] = a
    for name in ("xe", "ye", "co"):
        P[name][0] = 1.0
        P[name][3] = 2.5
    return U


def theta_s_faces(g, U, Cs=1.0):
    c = O.make_cfg(g, mu=1e-3, limiter=O.LIM_SMOOTH, Cs=Cs)
    _, fl, ts, _ = O.fe(c, U, 1e-6, want_theta=True)
    nfx = g.n2 * (g.n1 + 1)
    return ts[:nfx].reshape(g.n2, g.n1 + 1), ts[nfx:].reshape(g.n2 + 1, g.n1)


def test_theta_s_closed_form_with_divergence_and_curl():
    n1, n2 = 10, 9
    g = W.Grid(dim=2, n1=n1, n2=n2, x1=1.0, y1=0.9)
    dx, dy = g.dx, g.dy
    j, i = np.mgrid[0:n2, 0:n1].astype(float)
    I, J = i - 5.0, j - 4.0
    a, s, b = -0.02, 0.004, 0.03      # u = a I + s I^2 + b J
    cc, e, w = -0.04, -0.015, -0.003   # v = c I + e J + w J^2
    P0, al, be, ga = 1.0, 0.2, 0.3, 0.05  # p = P0 + al I^2 + be J^2 + ga I^2 J^2
    u = a * I + s * I ** 2 + b * J
    v = cc * I + e * J + w * J ** 2
    p = P0 + al * I ** 2 + be * J ** 2 + ga * I ** 2 * J ** 2
    r = 1.0 + 0.05 * ((i + 2 * j) % 3)
    U = state_from_cells(g, r, u, v, p)

    # closed forms per cell
    # f(I+1) - 2 f(I) + f(I-1) = 2 and f(I+1) + 2 f(I) + f(I-1) = 4 f(I) + 2
    # for f = I^2, so along x: 2 (al + ga J^2) and 4 p + 2 (al + ga J^2)
    cx, cy = al + ga * J ** 2, be + ga * I ** 2
    phi1x = abs(2 * cx) / abs(4 * p + 2 * cx)
    phi1y = abs(2 * cy) / abs(4 * p + 2 * cy)
    phi1 = np.maximum(phi1x, phi1y)
    div = (a + 2 * s * I) / dx + (e + 2 * w * J) / dy
    curl = cc / dx - b / dy
    phi2 = np.maximum(-div / np.sqrt(div ** 2 + curl ** 2 + 1e-13), 0.0)
    # the data exercise every part of the formula
    assert (phi1y > phi1x).any() and (phi1x > phi1y).any()
    assert (phi2 > 0).any() and (phi2 == 0).any()
    # without the curl, phi_2 would differ by more than 0.1 in many cells
    phi2_nocurl = np.maximum(-div / np.sqrt(div ** 2 + 1e-13), 0.0)
    assert ((phi2_nocurl - phi2) > 0.1).sum() > 20

    tx, ty = theta_s_faces(g, U)
    checked = 0
    # x-face (fi, fj) between cells (fi-1, fj) and (fi, fj); stencils that do
    # not wrap around the periodic box
    for fj in range(1, n2 - 1):
        for fi in range(2, n1 - 1):
            ph1 = max(phi1[fj, fi - 1], phi1[fj, fi])
            ph2 = max(phi2[fj, fi - 1], phi2[fj, fi])
            assert abs(tx[fj, fi] - np.exp(-ph1 * ph2)) < 1e-13, (fi, fj)
            checked += ph1 * ph2 > 0
    for fj in range(2, n2 - 1):
        for fi in range(1, n1 - 1):
            ph1 = max(phi1[fj - 1, fi], phi1[fj, fi])
            ph2 = max(phi2[fj - 1, fi], phi2[fj, fi])
            assert abs(ty[fj, fi] - np.exp(-ph1 * ph2)) < 1e-13, (fi, fj)
            checked += ph1 * ph2 > 0
    assert checked > 40
    # the face max matters: on some faces min and max of the product differ
    prods = [(min(phi1[fj, fi - 1], phi1[fj, fi]) * min(phi2[fj, fi - 1], phi2[fj, fi]),
              max(phi1[fj, fi - 1], phi1[fj, fi]) * max(phi2[fj, fi - 1], phi2[fj, fi]))
             for fj in range(1, n2 - 1) for fi in range(2, n1 - 1)]
    assert max(hi - lo for lo, hi in prods) > 1e-2


def test_theta_s_regularisation_inside_the_root():
    """no curl and div^2 = 1e-13: phi_2 = 1/sqrt(2) exactly, so
    theta^s = exp(-phi_1/sqrt(2)) with phi_1 from the x pressure curvature"""
    n1, n2 = 12, 6
    g = W.Grid(dim=2, n1=n1, n2=n2, x1=1.2, y1=0.6)
    dx = g.dx
    j, i = np.mgrid[0:n2, 0:n1].astype(float)
    I = i - 6.0
    slope = -np.sqrt(1e-13) * dx           # du/dx = -sqrt(1e-13)
    u = slope * I
    v = np.zeros_like(u)
    al = 0.2
    p = 1.0 + al * I ** 2                  # no y variation: phi_1 from x only
    U = state_from_cells(g, np.ones_like(u), u, v, p)
    phi1 = abs(2 * al) / (4.0 + al * (4 * I ** 2 + 2))
    Cs = 1.7
    tx, _ = theta_s_faces(g, U, Cs=Cs)
    for fj in range(n2):
        for fi in range(2, n1 - 1):
            ph1 = max(phi1[fj, fi - 1], phi1[fj, fi])
            ref = np.exp(-Cs * ph1 / np.sqrt(2.0))
            assert abs(tx[fj, fi] - ref) < 1e-9, (fi, fj)


def test_theta_s_is_one_under_pure_rotation():
    """a divergence-free rotation (u = -b J, v = c I) has phi_2 = 0 in every
    cell whatever the pressure curvature: theta^s = 1"""
    n1, n2 = 10, 10
    g = W.Grid(dim=2, n1=n1, n2=n2)
    j, i = np.mgrid[0:n2, 0:n1].astype(float)
    I, J = i - 5.0, j - 5.0
    u, v = -0.3 * J, 0.2 * I
    p = 1.0 + 0.4 * I ** 2 + 0.1 * J ** 2
    U = state_from_cells(g, np.ones_like(u), u, v, p)
    tx, ty = theta_s_faces(g, U)
    assert np.abs(tx[1:-1, 2:-2] - 1.0).max() == 0.0
    assert np.abs(ty[2:-2, 1:-1] - 1.0).max() == 0.0
