"""GPU checks of the mixed-precision 2D stage (AF_PREC_MIXED) against the FP64
oracle.  Its stencils, fluxes and residuals run in FP32; the density/pressure
blends, the cell-average update and the point-value update run in FP64.

Tolerance: a stage changes U by dt R with |dt R| ~ CFL |U|, and R is formed
from FP32 fluxes and stencils whose relative rounding is ~1e-7 (a few
operations of unit roundoff 6e-8), so one stage differs from the FP64 stage
by ~1e-8..1e-7 of the state's scale.  The per-stage bar below is 1e-5
relative to the scale of each compared quantity (the same metric as the FP64
parity tests), two orders above that estimate; run-level results state their
relative L1 difference.  Conservation of the cell averages is exact up to
FP64 round-off: every face flux is stored once and subtracted in FP64 by
both cells."""
import numpy as np
import pytest
import torch

import oracle as O
from parity import rel_errors
from paper_2609_29081_amd import af
from paper_2609_29081_amd import workloads as W

pytestmark = pytest.mark.gpu

GAMMA = 1.4
REL_TOL_MIXED = 1e-5


def mixed_solver(grid, **kw):
    return af.Solver(grid, precision=af.PREC_MIXED, **kw)


def stage_errors(grid, U, **kw):
    """worst relative error of the mixed stages against the oracle's, each
    stage started from the oracle's previous stage output"""
    cfg = O.make_cfg(grid, **kw)
    S = mixed_solver(grid, **kw)
    dt = O.dt(cfg, U)
    prev, worst = U, 0.0
    for k in range(3):
        fe, fl_ref = O.fe(cfg, prev, dt)
        if k == 0:
            ref = fe
        else:
            a, b = (0.75, 0.25) if k == 1 else (1.0 / 3.0, 2.0 / 3.0)
            ref = a * U + b * fe
        Ukd, Und = S.to_device(prev), S.to_device(U)
        out = torch.empty_like(Ukd)
        S.af_reset_flags()
        S.af_rk_stage(k, Und if k else None, Ukd, out, dt=dt)
        torch.cuda.synchronize()
        got, fl = out.cpu().numpy(), S.af_read_flags()
        assert fl == fl_ref, (k, fl, fl_ref)
        if fl_ref:
            break
        worst = max(worst, max(rel_errors(grid, got, ref).values()))
        prev = ref
    return worst


@pytest.mark.parametrize("case", ["vortex", "walls", "smallest_walls", "tube", "rarefaction",
                                  "rarefaction_pexact"])
def test_mixed_stages_close_to_fp64_oracle(case):
    if case == "vortex":
        g, f = W.vortex_wave_2d(48)
        kw = dict(mu=1e-3, Pr=0.72)
    elif case == "walls":
        g, f = W.random_smooth_2d(37, 22, seed=3, bc=(W.NOSLIP, W.OUTFLOW, W.SYMMETRY, W.NOSLIP),
                                  amp=0.15)
        kw = dict(mu=0.01, Pr=0.72)
    elif case == "smallest_walls":   # 4x4 cells: one tile, ghosts past every side
        g, f = W.random_smooth_2d(4, 4, seed=7, bc=(W.NOSLIP, W.SYMMETRY, W.SYMMETRY, W.NOSLIP),
                                  amp=0.1)
        kw = dict(mu=0.02, Pr=0.73)
    elif case == "tube":
        g, f = W.shock_tube_2d(48, 24, rho_left=3.0)
        kw = dict(mu=0.005, Pr=0.73)
    else:
        g, f = W.double_rarefaction(40, 24, speed=1.5)
        kw = dict(mu=1e-3, Pr=0.72)
        if case == "rarefaction_pexact":   # the pressure factor solved exactly
            kw["limiter"] = O.LIM_ALL | O.LIM_PEXACT
    U = W.make_state(g, f, GAMMA)
    worst = stage_errors(g, U, **kw)
    print(f"{case}: worst per-stage relative error {worst:.3e}")
    assert worst <= REL_TOL_MIXED


def test_mixed_conserves_cell_averages_exactly():
    g, f = W.vortex_wave_2d(64)
    U = W.make_state(g, f, GAMMA)
    S = mixed_solver(g, mu=1e-3, Pr=0.72)
    Ud = S.to_device(U)
    tot0 = g.split(U)["avg"].reshape(4, -1).sum(axis=1)
    st, n, t = S.af_run(Ud, 0.0, 1e30, 20, check_every=1)
    assert st == af.AF_OK and n == 20
    tot1 = g.split(Ud.cpu().numpy())["avg"].reshape(4, -1).sum(axis=1)
    scale = np.abs(g.split(U)["avg"]).reshape(4, -1).sum(axis=1)
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * scale), (tot1 - tot0) / scale


def test_mixed_run_l1_difference_and_positivity():
    # smooth run: relative L1 difference of the averages after 40 steps
    g, f = W.vortex_wave_2d(64)
    U = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, mu=1e-3, Pr=0.72)
    ref = U.copy()
    st, n, t_ref = O.run(cfg, ref, 0.0, 1e30, 40)
    S = mixed_solver(g, mu=1e-3, Pr=0.72)
    Ud = S.to_device(U)
    st, n, t = S.af_run(Ud, 0.0, 1e30, 40, check_every=1)
    assert st == af.AF_OK and n == 40
    got = Ud.cpu().numpy()
    A, B = g.split(got)["avg"], g.split(ref)["avg"]
    l1 = np.abs(A - B).sum() / np.abs(B).sum()
    print(f"vortex 64^2, 40 steps: relative L1 difference {l1:.3e}, t {t:.6g} vs {t_ref:.6g}")
    assert abs(t - t_ref) <= 1e-6 * t_ref
    assert l1 <= 1e-6
    # near vacuum: the blends in FP64 keep every DOF admissible
    g, f = W.double_rarefaction(48, 48, speed=2.0, angle=0.4)
    U = W.make_state(g, f, GAMMA)
    S = mixed_solver(g, mu=1e-3, Pr=0.72)
    Ud = S.to_device(U)
    st, n, t = S.af_run(Ud, 0.0, 1e30, 15, check_every=1)
    assert st == af.AF_OK and n == 15
    assert S.af_check_admissible(Ud) == 0


def test_mixed_full_size_shock_tube_two_steps():
    g, f = W.shock_tube_2d(1000, 500)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=0.005, Pr=0.73)
    cfg = O.make_cfg(g, **kw)
    ref = U.copy()
    st, n, t_ref = O.run(cfg, ref, 0.0, 1e30, 2)
    S = mixed_solver(g, **kw)
    Ud = S.to_device(U)
    st, n, t = S.af_run(Ud, 0.0, 1e30, 2, check_every=1)
    assert st == af.AF_OK and n == 2
    worst = max(rel_errors(g, Ud.cpu().numpy(), ref).values())
    print(f"shock tube 1000x500, 2 steps: worst relative error {worst:.3e}")
    assert worst <= REL_TOL_MIXED
    assert S.af_check_admissible(Ud) == 0


def test_mixed_cold_jet_stays_finite():
    """a sweep instance (768x384, Re 635, density ratio 190) whose early
    steps make a cold, fast jet where the diaphragm meets the bottom wall:
    internal energy a fraction of a percent of the total.  The point
    auxiliaries and low-order point values are taken from FP64 values, so
    the FP32 stencils never see a negative pressure; before that, the run
    ended with a non-finite state at step 80"""
    g, f, kw = W.shock_tube_sweep(64, seed=0)[3]
    assert (g.n1, g.n2) == (768, 384)
    S = mixed_solver(g, **kw)
    Ud = S.to_device(W.make_state(g, f, kw["gamma"]))
    st, n, t = S.af_run(Ud, 0.0, 1e30, 100, check_every=1)
    assert st == af.AF_OK and n == 100
    assert torch.isfinite(Ud).all()
    assert S.af_check_admissible(Ud) == 0


def test_exact_pressure_rule_runs_stay_admissible():
    """the receding rarefactions under the exact pressure rule, whose limited
    states sit at p = eps: 40 steps in FP64 and with FP32 stencils end with
    every DOF finite and admissible (the positivity of Sec. 3.4)"""
    g, f = W.double_rarefaction(40, 24, speed=1.5)
    U0 = W.make_state(g, f, GAMMA)
    kw = dict(mu=1e-3, Pr=0.72, limiter=af.LIM_ALL | af.LIM_PEXACT)
    for prec in (af.PREC_FP64, af.PREC_MIXED):
        S = af.Solver(g, precision=prec, **kw)
        Ud = S.to_device(U0)
        st, n, t = S.af_run(Ud, 0.0, 1e30, 40, check_every=1)
        assert st == af.AF_OK and n == 40, (prec, st, n)
        assert S.af_check_admissible(Ud) == 0
        assert np.isfinite(Ud.cpu().numpy()).all()
        print(f"precision {prec}: 40 steps to t = {t:.4e}")


def test_vortex_wave_two_hundred_steps_close_to_the_fp64_oracle():
    """the smooth vortex wave (64^2, mu = 1e-3) through 200 steps with FP32
    stencils beside the FP64 oracle's run: the FP32 rounding of each stage
    does not grow into more than the per-stage bar (measured 6.0e-8
    relative L1 and 2.9e-7 at worst, normwise; the final times, from CFL
    steps of slightly different averages, 1.7e-8 apart)"""
    g, f = W.vortex_wave_2d(64)
    U0 = W.make_state(g, f, GAMMA)
    kw = dict(mu=1e-3, Pr=0.72)
    S = mixed_solver(g, **kw)
    Ud = S.to_device(U0)
    st, n, t = S.af_run(Ud, 0.0, 1e30, 200, check_every=1)
    ref = U0.copy()
    sto, no, to = O.run(O.make_cfg(g, **kw), ref, 0.0, 1e30, 200)
    assert st == af.AF_OK and sto == 0 and n == no == 200
    assert t == pytest.approx(to, rel=1e-6)
    a = Ud.cpu().numpy()
    l1 = np.abs(a - ref).sum() / np.abs(ref).sum()
    worst = max(rel_errors(g, a, ref).values())
    print(f"vortex wave 64^2, FP32 stencils, 200 steps: relative L1 {l1:.3e}, worst {worst:.3e}")
    assert l1 <= 1e-6
    assert worst <= REL_TOL_MIXED
