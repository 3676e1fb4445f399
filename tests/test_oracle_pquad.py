"""Pins of the exact pressure rule of the density/pressure limiter (reading
R-pquad, switch LIM_PEXACT): theta^p is the largest blend t in [0, 1] with
p(U^L + s (U^T - U^L)) >= eps for every s <= t (Sec. 3.3), where the linear
rule takes the bound that the concavity of p gives.

* On random segments, 1D and 2D, near vacuum included, the oracle's theta^p
  equals the root that exact rational bisection finds for
  (gamma - 1)(E - |m|^2 / (2 rho)) = eps, to 1e-11.
* It is never below the linear rule's theta^p (concavity of p along a
  segment of positive density), and the pressure at it is eps.
* With p(U^L) at the 1e-13 floor the blend is 0, as under the linear rule.
* A segment from a dense state to a near-vacuum one (the crossing 1.4e-12
  from the far end) still lands on eps.
* Whole stages: the switch changes nothing where no pressure limiting acts
  (bit for bit), and where it acts each face's theta^rho theta^p is at least
  the linear rule's, the stage output stays admissible, and the wall-free
  stage conserves mass to round-off.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2609_29081_amd import workloads as W

GAMMA = 1.4


def _segment(rng, dim, near_vacuum):
    """an admissible U^L and a U^T of positive density whose pressure is
    negative (so the pressure limiter acts)"""
    nm = dim
    rL = rng.uniform(0.1, 2.0)
    uL = rng.uniform(-2.0, 2.0, nm)
    pL = 10.0 ** rng.uniform(-12.9, -11.0) if near_vacuum else 10.0 ** rng.uniform(-3.0, 0.3)
    rT = rng.uniform(0.05, 2.0)
    uT = rng.uniform(-3.0, 3.0, nm)
    pT = -(10.0 ** rng.uniform(-3.0, 0.0))
    def cons(r, u, p):
        return np.array([r, *(r * u), p / (GAMMA - 1.0) + 0.5 * r * float(u @ u)])
    return cons(rL, uL, pL), cons(rT, uT, pT)


def _q(UL, UT, s, g1, e):
    """(rho(s) (E(s) - e / g1) - |m(s)|^2 / 2) in exact rational arithmetic"""
    U = [Fraction(a) + s * (Fraction(b) - Fraction(a)) for a, b in zip(UL, UT)]
    m2 = sum(x * x for x in U[1:-1])
    return U[0] * (U[-1] - e / g1) - m2 / 2


def _bisect_root(UL, UT, eps):
    g1 = Fraction(GAMMA - 1.0)     # the same (gamma - 1) as the oracle's pressure
    e = Fraction(eps)
    lo, hi = Fraction(0), Fraction(1)
    assert _q(UL, UT, lo, g1, e) >= 0 > _q(UL, UT, hi, g1, e)
    for _ in range(90):
        mid = (lo + hi) / 2
        if _q(UL, UT, mid, g1, e) >= 0:
            lo = mid
        else:
            hi = mid
    return float(lo)


def _cfg(dim, limiter=O.LIM_ALL | O.LIM_PEXACT):
    g = W.Grid(dim=dim, n1=8, n2=8 if dim == 2 else 0)
    return O.make_cfg(g, limiter=limiter)


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("near_vacuum", [False, True])
def test_root_is_the_exact_crossing(dim, near_vacuum):
    rng = np.random.default_rng(11 + dim + 10 * near_vacuum)
    cfg = _cfg(dim)
    worst = 0.0
    for _ in range(60):
        UL, UT = _segment(rng, dim, near_vacuum)
        eps = min(1e-13, O.pressure(cfg, UL))
        th = O.theta_p_root(cfg, UL, UT, eps)
        ref = _bisect_root(UL, UT, eps)
        worst = max(worst, abs(th - ref))
        assert abs(th - ref) <= 1e-11, (UL, UT, th, ref)
    print(f"dim {dim}, near vacuum {near_vacuum}: worst |theta - exact root| {worst:.2e}")


@pytest.mark.parametrize("dim", [1, 2])
def test_root_not_below_the_linear_rule_and_pressure_at_eps(dim):
    rng = np.random.default_rng(5 + dim)
    cfg = _cfg(dim)
    for k in range(200):
        UL, UT = _segment(rng, dim, near_vacuum=(k % 4 == 0))
        pL, pT = O.pressure(cfg, UL), O.pressure(cfg, UT)
        eps = min(1e-13, pL)
        th = O.theta_p_root(cfg, UL, UT, eps)
        lin = O.theta(pL, pT, eps)
        assert 0.0 <= lin <= th <= 1.0
        p = O.pressure(cfg, UL + th * (UT - UL))
        scale = 1.0 + abs(UL[-1]) + abs(UT[-1])
        assert abs(p - eps) <= 1e-14 * scale, (p, eps)


def test_no_limiting_where_the_pressure_stays_above_eps():
    cfg = _cfg(2)
    UL = np.array([1.0, 0.3, -0.2, 2.5])
    UT = np.array([0.8, 0.1, 0.4, 1.9])
    assert O.pressure(cfg, UT) > 1e-13
    assert O.theta_p_root(cfg, UL, UT, 1e-13) == 1.0


def test_pressure_of_ul_at_the_floor_gives_zero():
    """p(U^L) at the 1e-13 floor (eps = p(U^L)): the blend is 0, as under the
    linear rule, even where the pressure would rise first along the segment
    and return to the floor further on"""
    cfg = _cfg(1)
    g1 = GAMMA - 1.0
    UL = np.array([1.0, 0.0, 1e-14 / g1])
    eps = min(1e-13, O.pressure(cfg, UL))
    # q(s) = rho (E - eps/g1) - m^2/2 = s - 2 s^2 with rho = 1, E = eps/g1 + s,
    # m = 2 s: the pressure rises, then crosses the floor again at s = 1/2
    UT = np.array([1.0, 2.0, 1e-14 / g1 + 1.0])
    assert O.pressure(cfg, UT) < 0.0
    assert O.theta_p_root(cfg, UL, UT, eps) == 0.0
    assert O.theta(eps, O.pressure(cfg, UT), eps) == 0.0


def test_dense_to_near_vacuum_segment_lands_on_eps():
    """a segment from a dense state to a near-vacuum one whose pressure is
    just below zero (from a shock-tube point update): the crossing lies
    1.4e-12 from the far end, where the pressure changes by about 1e3 per
    unit of the blend; the blend must still put the pressure at eps, not
    below (solving the quadratic about U^L put it at -1.3e-12)"""
    cfg = _cfg(2)
    UL = np.array([5.9171657912943427, 3.5634170000454102, -0.0081445259843001862,
                   10.813840360482907])
    UT = np.array([0.00044150857118543404, -0.001343933598765972, -0.00043192216630333135,
                   0.0022567106760020919])
    assert O.pressure(cfg, UT) < 0.0
    eps = 1e-13
    th = O.theta_p_root(cfg, UL, UT, eps)
    ref = _bisect_root(UL, UT, eps)
    assert 1.0 - th == pytest.approx(1.0 - ref, rel=1e-6)
    p = O.pressure(cfg, UL + th * (UT - UL))
    assert 0.9 * eps <= p <= 1.1e-12, p
    assert th >= O.theta(O.pressure(cfg, UL), O.pressure(cfg, UT), eps)


def _rarefaction_state(dim):
    if dim == 2:
        g, f = W.double_rarefaction(40, 24)
        kw = dict(mu=1e-3, Pr=0.72)
        nsteps = 2
    else:
        g, f = W.double_rarefaction(101)
        kw = dict(mu=0.0)
        nsteps = 5
    U = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, limiter=O.LIM_ALL, **kw)
    for _ in range(nsteps):
        assert O.step(cfg, U)[0] == 0
    return g, U, kw


@pytest.mark.parametrize("dim", [1, 2])
def test_stage_with_the_exact_rule(dim):
    g, U, kw = _rarefaction_state(dim)
    lin = O.make_cfg(g, limiter=O.LIM_ALL, **kw)
    ex = O.make_cfg(g, limiter=O.LIM_ALL | O.LIM_PEXACT, **kw)
    dt = O.dt(lin, U)
    a, fa, tsa, tpa = O.fe(lin, U, dt, want_theta=True)
    b, fb, tsb, tpb = O.fe(ex, U, dt, want_theta=True)
    # the pressure limiter acts on some faces, and the face states are the
    # same in both stages, so the exact rule's blend is never smaller
    act = tpa < 1.0
    assert act.sum() > 0
    assert np.all(tpb >= tpa - 1e-15)
    assert np.any(tpb[act] > tpa[act] + 1e-6)
    assert np.array_equal(tpb[~act], tpa[~act])
    assert not np.array_equal(a, b)
    # every DOF of the output admissible (density and pressure positive)
    assert fb == fa
    for V in g.split(b).values():
        m2 = sum(V[k] ** 2 for k in range(1, g.ncomp - 1))
        p = (GAMMA - 1.0) * (V[-1] - 0.5 * m2 / V[0])
        assert np.all(V[0] > 0) and np.all(p > 0)


def test_stage_with_the_exact_rule_conserves_on_a_periodic_grid():
    """the periodic double rarefaction along x (both axes periodic): the
    exact rule changes only theta, so the cell sums stay what they were"""
    g0, f = W.double_rarefaction(40, 24)
    g = W.Grid(dim=2, n1=g0.n1, n2=g0.n2, bc=(W.PERIODIC,) * 4)
    U = W.make_state(g, f, GAMMA)
    ex = O.make_cfg(g, limiter=O.LIM_ALL | O.LIM_PEXACT, mu=1e-3, Pr=0.72)
    for _ in range(2):
        assert O.step(ex, U)[0] == 0
    out, fl, ts, tp = O.fe(ex, U, O.dt(ex, U), want_theta=True)
    assert (tp < 1.0).sum() > 0
    s0 = g.split(U)["avg"].sum(axis=(1, 2))
    s1 = g.split(out)["avg"].sum(axis=(1, 2))
    assert np.allclose(s1, s0, rtol=0, atol=1e-11 * np.abs(s0).max())


def test_switch_is_inert_on_smooth_data():
    g, f = W.vortex_wave_2d(24)
    U = W.make_state(g, f, GAMMA)
    lin = O.make_cfg(g, limiter=O.LIM_ALL, mu=1e-3, Pr=0.72)
    ex = O.make_cfg(g, limiter=O.LIM_ALL | O.LIM_PEXACT, mu=1e-3, Pr=0.72)
    dt = O.dt(lin, U)
    a, fa = O.fe(lin, U, dt)
    b, fb = O.fe(ex, U, dt)
    assert fa == fb == 0
    assert np.array_equal(a, b)
