"""Pins of the oracle's positivity time-step bound (the theorem at the end of
Sec. 3.4): dt <= dx_l / (2 d max lambda_l) for the cell averages' LLF scheme
(the proposition on its intermediate states, Sec. 3.1) and the same on the
half lattice (spacing dx_l / 2) for the low-order point scheme, lambda being
bounded by the largest |u_l| + c plus the largest viscous coefficient b_l.

* On a uniform state the gradients vanish, b = 0, and the bound has a closed
  form: dx_l / (8 (|u_l| + c)) in 2D with both limiters (the point scheme's
  half spacing binds), dx_l / (4 (|u_l| + c)) with the cell limiter alone,
  dx / (4 (|u| + c)) in 1D; +infinity with neither low-order scheme in use.
* Taking max varrho + max b in place of the largest link lambda can only
  shrink the step, by at most half: half the per-link bound <= dt_pp <= the
  per-link bound (computed independently on the periodic half lattice).
* Under it the first forward-Euler stage raises no flag (all low-order cell
  and point states admissible) on hard data: a cold state rough at the
  lattice scale, a near-vacuum 1D Riemann problem and a 2D double
  rarefaction.
"""
import numpy as np
import pytest

import oracle as O
from paper_2609_29081_amd import workloads as W
from test_oracle_point_llf import half_lattice, link_lambda, llf_pieces, rough_cold_state

GAMMA = 1.4


@pytest.mark.parametrize("bc", [W.PERIODIC, W.NOSLIP])
def test_uniform_state_closed_form_2d(bc):
    g = W.Grid(dim=2, n1=14, n2=9, x1=1.4, y1=0.6, bc=(bc,) * 4)
    r, u, v, p = 1.3, (0.4 if bc == W.PERIODIC else 0.0), (-0.7 if bc == W.PERIODIC else 0.0), 0.9
    U = W.make_state(g, lambda x, y: (r + 0 * x, u + 0 * x, v + 0 * x, p + 0 * x), GAMMA)
    cs = np.sqrt(GAMMA * p / r)
    both = min(g.dx / (8 * (abs(u) + cs)), g.dy / (8 * (abs(v) + cs)))
    cell = min(g.dx / (4 * (abs(u) + cs)), g.dy / (4 * (abs(v) + cs)))
    c = O.make_cfg(g, mu=0.01)
    assert O.dt_pp(c, U) == pytest.approx(both, rel=1e-14)
    c = O.make_cfg(g, mu=0.01, limiter=O.LIM_PP | O.LIM_SMOOTH)
    assert O.dt_pp(c, U) == pytest.approx(cell, rel=1e-14)
    c = O.make_cfg(g, mu=0.01, limiter=O.LIM_SMOOTH | O.LIM_CENTRE)
    assert O.dt_pp(c, U) == np.inf


def test_uniform_state_closed_form_1d():
    g = W.Grid(dim=1, n1=20, x1=2.0)
    r, u, p = 0.8, -0.3, 1.7
    U = W.make_state(g, lambda x: (r + 0 * x, u + 0 * x, p + 0 * x), GAMMA)
    cs = np.sqrt(GAMMA * p / r)
    c = O.make_cfg(g, mu=0.02)
    assert O.dt_pp(c, U) == pytest.approx(g.dx / (4 * (abs(u) + cs)), rel=1e-14)


def test_between_half_and_all_of_the_per_link_bound():
    g, U = rough_cold_state(seed=11)
    mu, Pr = 0.05, 0.72
    H = half_lattice(g, U)
    _, _, ax, ay, bx, by = llf_pieces(g, H, mu, Pr)
    per_link = min(0.5 * g.dx / (4 * link_lambda(ax, bx, 1).max()),
                   0.5 * g.dy / (4 * link_lambda(ay, by, 0).max()))
    c = O.make_cfg(g, mu=mu, Pr=Pr, limiter=O.LIM_POINT)
    d = O.dt_pp(c, U)
    assert 0.5 * per_link <= d <= per_link * (1 + 1e-14)
    # on these data the two lambda forms differ
    assert d < per_link * (1 - 1e-6)


def hard_cases():
    g, U = rough_cold_state(seed=5)
    yield "rough cold 2D", g, U, dict(mu=0.05, Pr=0.72)
    g, f = W.leblanc_1d(200)
    yield "near-vacuum 1D", g, W.make_state(g, f, GAMMA), dict(mu=1e-3, Pr=0.75)
    g, f = W.double_rarefaction(32, 24, speed=3.0, angle=0.5)
    yield "double rarefaction 2D", g, W.make_state(g, f, GAMMA), dict(mu=0.01, Pr=0.72)


@pytest.mark.parametrize("case", list(range(3)))
def test_first_stage_admissible_under_the_bound(case):
    name, g, U, phys = list(hard_cases())[case]
    c = O.make_cfg(g, **phys)
    d = O.dt_pp(c, U)
    assert 0.0 < d < np.inf
    _, fl = O.fe(c, U, d)
    assert fl == 0, name
    # the low-order states alone stay admissible too (no flag, finite)
    c = O.make_cfg(g, limiter=O.LIM_LOWONLY | O.LIM_PP | O.LIM_POINT | O.LIM_CENTRE, **phys)
    out, fl = O.fe(c, U, d)
    assert fl == 0 and np.isfinite(out).all(), name
