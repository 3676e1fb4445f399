"""Pins of the oracle's SSP-RK54 (the five-stage, fourth-order SSP method
that Sec. 2.3 names): on a fixed grid, with the limiters off so that the
semi-discrete operator is smooth, the time error of RK54 falls as dt^4 and
that of SSP-RK3 as dt^3; one RK54 step from a constant state returns it
exactly; and RK54 with its halving keeps a near-vacuum state admissible."""
import numpy as np
import pytest

import oracle as O
from paper_2609_29081_amd import workloads as W

GAMMA = 1.4


def advance(cfg, U0, T, n):
    U = U0.copy()
    dt = T / n
    for k in range(n):
        st, dtu, h, fl = O.step(cfg, U, dt=dt, t=k * dt, t_final=1e30)
        assert st == 0 and h == 0 and dtu == dt
    return U


@pytest.mark.parametrize("rk,order", [(54, 4), (3, 3)])
def test_time_order_on_a_fixed_grid(rk, order):
    g, f = W.vortex_wave_2d(16)
    U0 = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, gamma=GAMMA, mu=1e-3, limiter=0, rk=rk)
    T = 0.03
    ref = advance(cfg, U0, T, 96)
    errs = [np.abs(advance(cfg, U0, T, n) - ref).max() for n in (3, 6, 12)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - order) < 0.35 for r in rates), (rk, errs, rates)


def test_constant_state_is_kept():
    g, f = W.random_smooth_2d(10, 9, seed=0, amp=0.0)
    U0 = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, gamma=GAMMA, mu=1e-3, rk=54, cfl_c=0.52, cfl_v=0.165)
    U = U0.copy()
    st, dtu, h, fl = O.step(cfg, U)
    assert st == 0 and dtu > 0
    assert np.abs(U - U0).max() <= 1e-14 * np.abs(U0).max()


def test_near_vacuum_steps_stay_admissible():
    g, f = W.double_rarefaction(40, 0, speed=2.0)
    U = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, gamma=GAMMA, mu=1e-3, rk=54, cfl_c=1.04, cfl_v=0.33)
    for _ in range(10):
        st, dtu, h, fl = O.step(cfg, U)
        assert st == 0
    P = g.split(U)
    for name in P:
        r = P[name][0]
        p = (GAMMA - 1.0) * (P[name][2] - 0.5 * P[name][1] ** 2 / r)
        assert r.min() > 0 and p.min() > 0
