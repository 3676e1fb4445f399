"""GPU (HIP, through the C ABI) vs FP64 CPU oracle, element by element.

Every case feeds both sides the same seeded synthetic input and compares
each DOF array and component to 1e-12 relative (FP64 path).  Grids are
chosen so that the launches have ragged last blocks and so that every
boundary kind, the limiter switches and the degenerate cases (smallest
grid, mu = 0, limiter inactive/active, step halving) are exercised.
"""
import numpy as np
import pytest
import torch

import oracle as O
from parity import assert_close, assert_close_pointwise
from paper_2609_29081_amd import af
from paper_2609_29081_amd import workloads as W

pytestmark = pytest.mark.gpu

GAMMA = 1.4


def solver_for(grid, **kw):
    return af.Solver(grid, **kw)


def gpu_stage(S, k, Un, Uk, dt):
    Ukd = S.to_device(Uk)
    Und = S.to_device(Un) if Un is not None else None
    out = torch.empty_like(Ukd)
    S.af_reset_flags()
    S.af_rk_stage(k, Und, Ukd, out, dt=dt)
    torch.cuda.synchronize()
    return out.cpu().numpy(), S.af_read_flags()


def oracle_stage(cfg, k, Un, Uk, dt):
    fe, fl = O.fe(cfg, Uk, dt)
    if k == 0:
        return fe, fl
    a, b = (0.75, 0.25) if k == 1 else (1.0 / 3.0, 2.0 / 3.0)
    return a * Un + b * fe, fl


def check_stages(grid, U, dt=None, pointwise=None, **kw):
    """the three stages of one step, each from the oracle's previous stage
    output, compared element by element.  A stage whose low-order states are
    flagged is one the step rejects (and redoes with dt/2): there the flags
    must agree, the values are not compared (a state that crossed rho = 0
    switches its blend parameter to 0, a discontinuous decision) and the
    comparison ends, since no later stage ever starts from such an output."""
    cfg = O.make_cfg(grid, **kw)
    S = solver_for(grid, **kw)
    if dt is None:
        dt = O.dt(cfg, U)
    prev = U
    worst = 0.0
    for k in range(3):
        ref, fl_ref = oracle_stage(cfg, k, U, prev, dt)
        got, fl_gpu = gpu_stage(S, k, U if k else None, prev, dt)
        assert fl_gpu == fl_ref, (k, fl_gpu, fl_ref)
        if fl_ref != 0:
            break
        worst = max(worst, assert_close(grid, got, ref, what=f"stage {k}"))
        if pointwise is not None:
            assert_close_pointwise(grid, got, ref, pointwise, what=f"stage {k}")
        prev = ref
    return worst


def accepted_dt(cfg, U):
    """time step the oracle's step would accept from U (after any halving)"""
    V = U.copy()
    st, dtu, h, fl = O.step(cfg, V)
    assert st == 0
    return dtu


# ---------------------------------------------------------------------------
# 2D stages
# ---------------------------------------------------------------------------
def test_stage_2d_vortex_periodic():
    g, f = W.vortex_wave_2d(40)
    check_stages(g, W.make_state(g, f, GAMMA), mu=1e-3, Pr=0.72)


@pytest.mark.parametrize("bc", [(W.NOSLIP,) * 4, (W.SYMMETRY,) * 4, (W.OUTFLOW,) * 4,
                                (W.PERIODIC, W.PERIODIC, W.NOSLIP, W.SYMMETRY),
                                (W.NOSLIP, W.OUTFLOW, W.PERIODIC, W.PERIODIC)])
def test_stage_2d_boundaries_nonsquare(bc):
    g, f = W.random_smooth_2d(37, 29, seed=5, bc=bc, x1=1.3, y1=0.7, amp=0.15)
    check_stages(g, W.make_state(g, f, GAMMA), mu=0.02, Pr=0.73)


def test_stage_2d_shock_tube_smoothness_active():
    g, f = W.shock_tube_2d(60, 30)
    U = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, mu=0.005, Pr=0.73)
    for _ in range(3):      # let the diaphragm spread
        assert O.step(cfg, U)[0] == 0
    out, fl, ts, tp = O.fe(cfg, U, O.dt(cfg, U), want_theta=True)
    assert ts.min() < 0.5
    check_stages(g, U, pointwise=1e-11, mu=0.005, Pr=0.73)


@pytest.mark.parametrize("angle", [0.0, 0.5])
@pytest.mark.parametrize("limiter", [O.LIM_PP | O.LIM_POINT | O.LIM_CENTRE, O.LIM_ALL])
def test_stage_2d_density_pressure_limiting_active(angle, limiter):
    """receding rarefactions: theta^rho theta^p strictly inside (0,1) on some
    faces, and (at the larger angle) flagged low-order states"""
    g, f = W.double_rarefaction(40, 24, angle=angle)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=1e-3, Pr=0.72, limiter=limiter)
    cfg = O.make_cfg(g, **kw)
    for _ in range(2):
        assert O.step(cfg, U)[0] == 0
    dt = accepted_dt(cfg, U)
    out, fl, ts, tp = O.fe(cfg, U, dt, want_theta=True)
    assert fl == 0
    if angle == 0.0:
        assert ((tp > 0) & (tp < 1)).sum() > 0
    check_stages(g, U, dt=dt, **kw)
    # and at the CFL step, where the low-order states are flagged
    check_stages(g, U, **kw)


@pytest.mark.parametrize("angle", [0.0, 0.5])
def test_stage_2d_exact_pressure_rule(angle):
    """the pressure factor solved exactly (LIM_PEXACT) on the receding
    rarefactions: it acts (the oracle's output differs from the linear
    rule's) and the GPU follows it"""
    g, f = W.double_rarefaction(40, 24, angle=angle)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=1e-3, Pr=0.72, limiter=O.LIM_ALL | O.LIM_PEXACT)
    cfg = O.make_cfg(g, **kw)
    for _ in range(2):
        assert O.step(cfg, U)[0] == 0
    dt = accepted_dt(cfg, U)
    lin = O.fe(O.make_cfg(g, mu=1e-3, Pr=0.72), U, dt)[0]
    assert not np.array_equal(O.fe(cfg, U, dt)[0], lin)
    check_stages(g, U, dt=dt, **kw)
    check_stages(g, U, **kw)


def test_stage_1d_exact_pressure_rule():
    g, f = W.double_rarefaction(101)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=0.0, limiter=O.LIM_PP | O.LIM_POINT | O.LIM_CENTRE | O.LIM_PEXACT)
    cfg = O.make_cfg(g, **kw)
    for _ in range(5):
        assert O.step(cfg, U)[0] == 0
    dt = O.dt(cfg, U)
    lin = O.fe(O.make_cfg(g, mu=0.0, limiter=O.LIM_PP | O.LIM_POINT | O.LIM_CENTRE), U, dt)[0]
    assert not np.array_equal(O.fe(cfg, U, dt)[0], lin)
    check_stages(g, U, **kw)


def test_steps_exact_pressure_rule_match_oracle():
    """five steps of the 2D receding rarefactions under LIM_PEXACT: the
    same time steps and halvings as the oracle, and the same state"""
    g, f = W.double_rarefaction(40, 24, angle=0.5)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=1e-3, Pr=0.72, limiter=O.LIM_ALL | O.LIM_PEXACT)
    cfg = O.make_cfg(g, **kw)
    S = solver_for(g, **kw)
    Ud = S.to_device(U)
    for n in range(5):
        st, dtu, h, fl = O.step(cfg, U)
        stg, dtg, hg = S.af_step(Ud)
        assert st == 0 and stg == af.AF_OK
        assert hg == h and dtg == pytest.approx(dtu, rel=1e-12), n
    assert_close(g, Ud.cpu().numpy(), U, what="five steps under the exact pressure rule")


def test_stage_1d_density_pressure_limiting_active():
    g, f = W.double_rarefaction(101)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=0.0, limiter=O.LIM_PP | O.LIM_POINT | O.LIM_CENTRE)
    cfg = O.make_cfg(g, **kw)
    for _ in range(5):
        assert O.step(cfg, U)[0] == 0
    out, fl, ts, tp = O.fe(cfg, U, O.dt(cfg, U), want_theta=True)
    assert ((tp > 0) & (tp < 1)).sum() > 0
    check_stages(g, U, **kw)


@pytest.mark.parametrize("limiter", [0, O.LIM_SMOOTH, O.LIM_PP, O.LIM_POINT, O.LIM_CENTRE,
                                     O.LIM_LOWONLY, O.LIM_LOWONLY | O.LIM_PP,
                                     O.LIM_LOWONLY | O.LIM_POINT])
def test_stage_2d_limiter_switches(limiter):
    """every switch on a mild shock tube (density ratio 2.5), where even the
    unlimited scheme keeps every state admissible"""
    g, f = W.shock_tube_2d(24, 16, rho_left=3.0)
    U = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, mu=0.005, Pr=0.73)
    assert O.step(cfg, U)[0] == 0
    check_stages(g, U, mu=0.005, Pr=0.73, limiter=limiter)


@pytest.mark.parametrize("bc", [(W.NOSLIP, W.SYMMETRY, W.SYMMETRY, W.NOSLIP),
                                (W.PERIODIC, W.PERIODIC, W.NOSLIP, W.OUTFLOW),
                                (W.OUTFLOW, W.NOSLIP, W.PERIODIC, W.PERIODIC)])
def test_stage_2d_smallest_grid_every_side_kind(bc):
    """the smallest grid (4x4 cells, one tile): ghost centres beyond every
    non-periodic side, whose images lie one and two cells from the side"""
    g, f = W.random_smooth_2d(4, 4, seed=7, bc=bc, amp=0.1)
    check_stages(g, W.make_state(g, f, GAMMA), mu=0.02, Pr=0.73)


def test_stage_2d_inviscid_and_smallest_grid():
    g, f = W.random_smooth_2d(4, 4, seed=2, bc=(W.OUTFLOW,) * 4, amp=0.1)
    check_stages(g, W.make_state(g, f, GAMMA), mu=0.0)
    g, f = W.random_smooth_2d(5, 4, seed=3, amp=0.1)
    check_stages(g, W.make_state(g, f, GAMMA), mu=0.01)


# ---------------------------------------------------------------------------
# 1D stages
# ---------------------------------------------------------------------------
def test_stage_1d_density_wave():
    g, f = W.density_wave_1d(128)
    check_stages(g, W.make_state(g, f, GAMMA), mu=1e-3, Pr=0.72, cfl_v=0.15)


def test_stage_1d_near_vacuum_limiting():
    g, f = W.leblanc_1d(203)
    U = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, mu=1e-5, Pr=0.75, cfl_v=0.15)
    for _ in range(3):
        assert O.step(cfg, U)[0] == 0
    check_stages(g, U, mu=1e-5, Pr=0.75, cfl_v=0.15)


@pytest.mark.parametrize("bc", [W.NOSLIP, W.SYMMETRY])
def test_stage_1d_walls(bc):
    g = W.Grid(dim=1, n1=45, bc=(bc, W.OUTFLOW, 0, 0))
    U = W.make_state(g, lambda x: (1 + 0.3 * np.exp(-40 * (x - 0.3) ** 2), 0.2 * np.sin(3 * x),
                                   1 + 0.2 * np.cos(5 * x)), GAMMA)
    check_stages(g, U, mu=0.01, Pr=0.72, cfl_v=0.15)


# ---------------------------------------------------------------------------
# CFL step, full steps with halving, runs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["vortex", "tube", "wave1d"])
def test_cfl_dt(case):
    if case == "vortex":
        g, f = W.vortex_wave_2d(33)
        kw = dict(mu=1e-3)
    elif case == "tube":
        g, f = W.shock_tube_2d(50, 25)
        kw = dict(mu=0.005, Pr=0.73)
    else:
        g, f = W.density_wave_1d(64)
        kw = dict(mu=1e-3, cfl_v=0.15)
    U = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, **kw)
    S = solver_for(g, **kw)
    d = S.af_cfl_dt(S.to_device(U), 0.0, 1e30)
    torch.cuda.synchronize()
    assert d.item() == pytest.approx(O.dt(cfg, U), rel=1e-14)
    d = S.af_cfl_dt(S.to_device(U), 0.3, 0.3 + 1e-7)
    assert d.item() == pytest.approx(1e-7, rel=1e-8)


def test_steps_2d_shock_tube():
    g, f = W.shock_tube_2d(48, 24)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=0.005, Pr=0.73)
    cfg = O.make_cfg(g, **kw)
    S = solver_for(g, **kw)
    Ud = S.to_device(U)
    t = 0.0
    for s in range(8):
        st, dtu, h, fl = O.step(cfg, U, 0.0, t)
        stg, dtg, hg = S.af_step(Ud, 0.0, t)
        assert st == 0 and stg == af.AF_OK and h == hg
        assert dtg == pytest.approx(dtu, rel=1e-13)
        t += dtu
        got = Ud.cpu().numpy()
        assert_close(g, got, U, tol=1e-12 * (s + 1), what=f"step {s}")
        assert_close_pointwise(g, got, U, tol=1e-11 * (s + 1), what=f"step {s}")


@pytest.mark.parametrize("mu,limiter", [(0.0, O.LIM_ALL), (1e-5, O.LIM_ALL),
                                        (0.0, O.LIM_ALL | O.LIM_PEXACT)])
def test_leblanc_runs_to_the_end_with_the_oracle(mu, limiter):
    """the paper's 1D LeBlanc problem (800 cells, outflow, near vacuum right
    of the diaphragm) to t = 0.4, inviscid and with mu = 1e-5, Pr = 0.75, and
    inviscid under the exact pressure rule (which moves the final state by
    2e-5 there): the same number of steps as the oracle's whole run, every
    DOF admissible, and the final states equal to the FP64 bar"""
    g, f = W.leblanc_1d(800)
    U0 = W.make_state(g, f, GAMMA)
    S = solver_for(g, mu=mu, Pr=0.75, limiter=limiter)
    Ud = S.to_device(U0)
    st, n, t = S.af_run(Ud, 0.0, 0.4, 10 ** 7, check_every=1)
    assert st == af.AF_OK and t == pytest.approx(0.4, rel=1e-15)
    assert S.af_check_admissible(Ud) == 0
    ref = U0.copy()
    sto, no, to = O.run(O.make_cfg(g, mu=mu, Pr=0.75, limiter=limiter), ref, 0.0, 0.4)
    assert sto == 0 and no == n
    worst = assert_close(g, Ud.cpu().numpy(), ref, tol=1e-12,
                         what=f"LeBlanc mu={mu} limiter={limiter}, t=0.4")
    print(f"LeBlanc mu={mu} limiter={limiter}: {n} steps, worst relative error {worst:.3e}")


@pytest.mark.parametrize("angle,mu,steps", [(0.0, 0.0, 0), (0.5, 0.0, 0), (0.5, 1e-3, 200)])
def test_receding_rarefactions_whole_run_with_the_oracle(angle, mu, steps):
    """2D receding rarefactions (a near-vacuum centre, the density and
    pressure limiting acting every step) run through af_run beside the
    oracle's own run: inviscid to t = 0.1, or 200 viscous steps; the same
    steps and final time, every DOF admissible, the final states within
    the FP64 bar, which for the viscous run grows with the steps (1e-12 per
    four steps: rounding differences are carried from step to step, and
    near vacuum the viscous terms, which scale as mu / rho, amplify them;
    measured 5e-15 and 6e-15 inviscid, 1.6e-11 after the 200 viscous
    steps)"""
    g, f = W.double_rarefaction(40, 24, speed=2.0, angle=angle)
    U0 = W.make_state(g, f, GAMMA)
    kw = dict(mu=mu, Pr=0.72)
    tf, ms = (0.1, 10 ** 6) if steps == 0 else (1e30, steps)
    S = solver_for(g, **kw)
    Ud = S.to_device(U0)
    st, n, t = S.af_run(Ud, 0.0, tf, ms, check_every=1)
    ref = U0.copy()
    sto, no, to = O.run(O.make_cfg(g, **kw), ref, 0.0, tf, ms)
    assert st == af.AF_OK and sto == 0 and n == no
    assert t == pytest.approx(to, rel=1e-12)
    assert S.af_check_admissible(Ud) == 0
    tol = 1e-12 if mu == 0.0 else 1e-12 * n / 4
    worst = assert_close(g, Ud.cpu().numpy(), ref, tol=tol,
                         what=f"rarefactions angle={angle} mu={mu}, {n} steps")
    print(f"rarefactions angle={angle} mu={mu}: {n} steps to t={t:.4g}, worst {worst:.3e}")


def test_vortex_wave_two_hundred_steps_with_the_oracle():
    """the smooth periodic vortex wave (64^2, mu = 1e-3) through 200 steps of
    af_run beside the oracle's run: the same final time, and the final
    states within the FP64 bar of single stages (smooth data: rounding
    differences are not amplified from step to step)"""
    g, f = W.vortex_wave_2d(64)
    U0 = W.make_state(g, f, GAMMA)
    kw = dict(mu=1e-3, Pr=0.72)
    S = solver_for(g, **kw)
    Ud = S.to_device(U0)
    st, n, t = S.af_run(Ud, 0.0, 1e30, 200, check_every=1)
    ref = U0.copy()
    sto, no, to = O.run(O.make_cfg(g, **kw), ref, 0.0, 1e30, 200)
    assert st == af.AF_OK and sto == 0 and n == no == 200
    assert t == pytest.approx(to, rel=1e-12)
    worst = assert_close(g, Ud.cpu().numpy(), ref, tol=1e-12, what="vortex wave 64^2, 200 steps")
    print(f"vortex wave 64^2: 200 steps to t={t:.4g}, worst relative error {worst:.3e}")


def test_halving_matches_oracle():
    g, f = W.leblanc_1d(160)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=0.0, Pr=0.75)
    cfg = O.make_cfg(g, **kw)
    S = solver_for(g, **kw)
    Ud = S.to_device(U)
    big = 40 * O.dt(cfg, U)
    st, dtu, h, fl = O.step(cfg, U, big)
    stg, dtg, hg = S.af_step(Ud, big)
    assert st == 0 and stg == af.AF_OK
    assert h >= 1 and hg == h and dtg == dtu
    assert_close(g, Ud.cpu().numpy(), U, what="halved step")


def test_halving_exhausted_restores_state():
    g, f = W.leblanc_1d(100)
    U = W.make_state(g, f, GAMMA)
    S = solver_for(g, mu=0.0, Pr=0.75, max_halvings=0)
    Ud = S.to_device(U)
    st, dtu, h = S.af_step(Ud, 300 * O.dt(O.make_cfg(g, mu=0.0, Pr=0.75), U))
    assert st == af.AF_E_PP
    assert np.array_equal(Ud.cpu().numpy(), U)


@pytest.mark.parametrize("check_every", [1, 64])
def test_run_1d_density_wave_to_t01(check_every):
    """the small 1D workload end to end: periodic, N=128, SSP-RK3, t=0.1"""
    g, f = W.density_wave_1d(128)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=1e-3, Pr=0.72, cfl_c=0.2, cfl_v=0.15)
    cfg = O.make_cfg(g, **kw)
    S = solver_for(g, **kw)
    Ud = S.to_device(U)
    st, ns, t = O.run(cfg, U, 0.0, 0.1)
    stg, nsg, tg = S.af_run(Ud, 0.0, 0.1, 1 << 30, check_every=check_every)
    assert st == 0 and stg == af.AF_OK and ns == nsg
    assert tg == pytest.approx(t, rel=1e-13) and t == pytest.approx(0.1, rel=1e-14)
    assert_close(g, Ud.cpu().numpy(), U, tol=1e-11, what="run to t=0.1")


@pytest.mark.parametrize("check_every", [1, 6])
def test_run_rollback_path(check_every):
    """a block whose flags rise is redone step by step with halving"""
    g, f = W.leblanc_1d(120)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=1e-5, Pr=0.75, cfl_v=0.15)
    cfg = O.make_cfg(g, **kw)
    S = solver_for(g, **kw)
    Ud = S.to_device(U)
    t = 0.0
    for _ in range(6):
        st, dtu, h, fl = O.step(cfg, U, 0.0, t)
        t += dtu
    stg, nsg, tg = S.af_run(Ud, 0.0, 1e30, 6, check_every=check_every)
    assert stg == af.AF_OK and nsg == 6
    assert tg == pytest.approx(t, rel=1e-12)
    assert_close(g, Ud.cpu().numpy(), U, tol=1e-10, what="run with rollback")


def test_full_size_shock_tube_steps():
    """the headline workload at its full size (1000 x 500), launched exactly as
    the benchmark launches it, against the oracle over two whole steps"""
    g, f = W.shock_tube_2d(1000, 500)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=0.005, Pr=0.73, cfl_c=0.2, cfl_v=0.05)
    cfg = O.make_cfg(g, **kw)
    S = solver_for(g, **kw)
    Ud = S.to_device(U)
    t = 0.0
    for _ in range(2):
        st, dtu, h, fl = O.step(cfg, U, 0.0, t)
        assert st == 0
        t += dtu
    stg, nsg, tg, att = S.af_run_graph(Ud, 0.0, 1e30, 2)
    assert stg == af.AF_OK and nsg == 2
    got = Ud.cpu().numpy()
    assert_close(g, got, U, tol=2e-12, what="full-size shock tube")
    assert_close_pointwise(g, got, U, tol=2e-11, what="full-size shock tube")
