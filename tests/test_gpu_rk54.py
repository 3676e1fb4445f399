"""GPU parity of SSP-RK54 stepping (af_params.rk = 54) against the oracle's
orc_step with rk = 54: the same five forward-Euler stages with their
fractions of dt, the shared fourth-stage evaluation and the two state
combinations, under the same halving rule.  Both sides are FP64; the bar is
the FP64 parity bar per step (1e-12 relative, growing with the number of
steps compared), dt and halvings exactly."""
import numpy as np
import pytest
import torch

import oracle as O
from parity import assert_close
from paper_2609_29081_amd import af
from paper_2609_29081_amd import workloads as W

pytestmark = pytest.mark.gpu

GAMMA = 1.4
RK54_2D = dict(cfl_c=0.52, cfl_v=0.165, rk=54)
RK54_1D = dict(cfl_c=1.04, cfl_v=0.33, rk=54)


def cases():
    out = []
    g, f = W.vortex_wave_2d(24)
    out.append(("vortex_2d", g, W.make_state(g, f, GAMMA), dict(mu=1e-3, Pr=0.72, **RK54_2D)))
    g, f = W.shock_tube_2d(48, 24)
    out.append(("shock_tube_2d", g, W.make_state(g, f, GAMMA), dict(mu=0.005, Pr=0.73, **RK54_2D)))
    g, f = W.random_smooth_2d(19, 23, seed=7, bc=(W.NOSLIP, W.OUTFLOW, W.SYMMETRY, W.NOSLIP),
                              amp=0.15)
    out.append(("walls_2d", g, W.make_state(g, f, GAMMA), dict(mu=0.01, Pr=0.72, **RK54_2D)))
    g, f = W.density_wave_1d(64)
    out.append(("density_wave_1d", g, W.make_state(g, f, GAMMA), dict(mu=1e-3, Pr=0.72, **RK54_1D)))
    g, f = W.leblanc_1d(120)
    out.append(("leblanc_1d", g, W.make_state(g, f, GAMMA), dict(mu=1e-5, Pr=0.75, **RK54_1D)))
    return out


@pytest.mark.parametrize("case", cases(), ids=lambda c: c[0])
def test_rk54_steps_match_the_oracle(case):
    name, g, U, kw = case
    cfg = O.make_cfg(g, gamma=GAMMA, **kw)
    S = af.Solver(g, gamma=GAMMA, **kw)
    Ud = S.to_device(U)
    t = 0.0
    halved = 0
    for s in range(5):
        st, dtu, h, fl = O.step(cfg, U, 0.0, t)
        stg, dtg, hg = S.af_step(Ud, 0.0, t)
        assert st == 0 and stg == af.AF_OK and hg == h, (name, s, h, hg)
        assert dtg == pytest.approx(dtu, rel=1e-13)
        halved += h
        t += dtu
        assert_close(g, Ud.cpu().numpy(), U, tol=1e-12 * (s + 1), what=f"{name} step {s}")


def test_rk54_halving_matches_the_oracle():
    g, f = W.leblanc_1d(160)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=0.0, Pr=0.75, **RK54_1D)
    cfg = O.make_cfg(g, gamma=GAMMA, **kw)
    S = af.Solver(g, gamma=GAMMA, **kw)
    Ud = S.to_device(U)
    big = 40 * O.dt(cfg, U)
    st, dtu, h, fl = O.step(cfg, U, big)
    stg, dtg, hg = S.af_step(Ud, big)
    assert st == 0 and stg == af.AF_OK
    assert h >= 1 and hg == h and dtg == dtu
    assert_close(g, Ud.cpu().numpy(), U, what="halved RK54 step")


@pytest.mark.parametrize("check_every", [1, 4])
def test_rk54_run_matches_the_oracle(check_every):
    """af_run's device-side steps (the fourth buffer in the rotation, the
    stage steps as device scalars) against the oracle's steps"""
    g, f = W.shock_tube_2d(40, 20, rho_left=60.0)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=0.005, Pr=0.73, **RK54_2D)
    cfg = O.make_cfg(g, gamma=GAMMA, **kw)
    S = af.Solver(g, gamma=GAMMA, **kw)
    Ud = S.to_device(U)
    st, ns, t = O.run(cfg, U, 0.0, 1e30, 7)
    stg, nsg, tg = S.af_run(Ud, 0.0, 1e30, 7, check_every=check_every)
    assert st == 0 and stg == af.AF_OK and ns == nsg == 7
    assert tg == pytest.approx(t, rel=1e-12)
    assert_close(g, Ud.cpu().numpy(), U, tol=1e-11, what=f"RK54 run, check_every {check_every}")


def test_rk54_mixed_precision_is_near_the_fp64_oracle():
    g, f = W.vortex_wave_2d(24)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=1e-3, Pr=0.72, **RK54_2D)
    cfg = O.make_cfg(g, gamma=GAMMA, **kw)
    S = af.Solver(g, gamma=GAMMA, precision=af.PREC_MIXED, **kw)
    Ud = S.to_device(U)
    dt = O.dt(cfg, U)
    for s in range(3):
        O.step(cfg, U, dt, s * dt)
        S.af_step(Ud, dt, s * dt)
    assert_close(g, Ud.cpu().numpy(), U, tol=1e-5, what="mixed RK54")
