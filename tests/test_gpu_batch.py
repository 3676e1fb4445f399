"""GPU checks of batches (af_batch_*): many independent 2D instances whose
stages run as one persistent launch per stage, each instance with its own
CFL time step and its own step halving decided on the device.  The batch
must reproduce, bit for bit, what af_run gives for each instance alone (the
same tile arithmetic, the same exact max-reductions for dt, the same
decisions), with and without HIP-graph replay, in both precisions; and a
small batch is checked against the FP64 oracle directly."""
import numpy as np
import pytest
import torch

import oracle as O
from parity import assert_close
from paper_2609_29081_amd import af
from paper_2609_29081_amd import workloads as W

pytestmark = pytest.mark.gpu

GAMMA = 1.4


def instances():
    """heterogeneous instances: sizes, boundaries, viscosities, a shock tube
    that halves its steps and a smooth periodic field that does not"""
    out = []
    g, f = W.shock_tube_2d(40, 20, rho_left=60.0)
    out.append((g, f, dict(mu=0.005, Pr=0.73)))
    g, f = W.vortex_wave_2d(24)
    out.append((g, f, dict(mu=1e-3, Pr=0.72)))
    g, f = W.random_smooth_2d(19, 33, seed=5, bc=(W.NOSLIP, W.OUTFLOW, W.SYMMETRY, W.NOSLIP),
                              amp=0.15)
    out.append((g, f, dict(mu=0.01, Pr=0.72)))
    g, f = W.shock_tube_2d(70, 35, rho_left=120.0)
    out.append((g, f, dict(mu=0.002, Pr=0.73)))
    g, f = W.double_rarefaction(30, 26, speed=1.5, angle=0.3)
    out.append((g, f, dict(mu=1e-3, Pr=0.72)))
    return out


def run_single(g, f, kw, steps, precision):
    S = af.Solver(g, precision=precision, **kw)
    U = S.to_device(W.make_state(g, f, GAMMA))
    st, n, t = S.af_run(U, 0.0, 1e30, steps, check_every=1)
    assert st == af.AF_OK and n == steps
    return U.cpu().numpy(), t


@pytest.mark.parametrize("precision,use_graph,aps", [(af.PREC_FP64, False, 4),
                                                     (af.PREC_FP64, True, 3),
                                                     (af.PREC_FP64, False, 1),
                                                     (af.PREC_MIXED, True, 4)])
def test_batch_reproduces_single_runs(precision, use_graph, aps):
    steps = 6
    insts = instances()
    solvers = [af.Solver(g, precision=precision, **kw) for g, f, kw in insts]
    states = [S.to_device(W.make_state(g, f, GAMMA)) for S, (g, f, kw) in zip(solvers, insts)]
    B = af.Batch(solvers)
    st, n, t, att = B.af_batch_run(states, 0.0, 1e30, steps, attempts_per_slot=aps,
                                   use_graph=use_graph)
    assert st == [af.AF_OK] * len(insts)
    assert n == [steps] * len(insts)
    assert max(att) > steps  # at least one instance halved a step
    for (g, f, kw), U, ti in zip(insts, states, t):
        ref, tr = run_single(g, f, kw, steps, precision)
        assert ti == tr
        assert np.array_equal(U.cpu().numpy(), ref)


@pytest.mark.parametrize("precision", [af.PREC_FP64, af.PREC_MIXED])
def test_batch_with_per_instance_pressure_rules(precision):
    """instances under the exact pressure rule (AF_LIM_PEXACT) beside
    instances under the linear one, in one batch: each reproduces its own
    single run bit for bit"""
    steps = 5
    insts = [(g, f, dict(kw, limiter=af.LIM_ALL | (af.LIM_PEXACT if k % 2 == 0 else 0)))
             for k, (g, f, kw) in enumerate(instances())]
    solvers = [af.Solver(g, precision=precision, **kw) for g, f, kw in insts]
    states = [S.to_device(W.make_state(g, f, GAMMA)) for S, (g, f, kw) in zip(solvers, insts)]
    st, n, t, att = af.Batch(solvers).af_batch_run(states, 0.0, 1e30, steps)
    assert st == [af.AF_OK] * len(insts) and n == [steps] * len(insts)
    for (g, f, kw), U, ti in zip(insts, states, t):
        ref, tr = run_single(g, f, kw, steps, precision)
        assert ti == tr
        assert np.array_equal(U.cpu().numpy(), ref)


def test_batch_matches_the_oracle():
    insts = instances()[1:3]
    solvers = [af.Solver(g, **kw) for g, f, kw in insts]
    states = [S.to_device(W.make_state(g, f, GAMMA)) for S, (g, f, kw) in zip(solvers, insts)]
    B = af.Batch(solvers)
    st, n, t, att = B.af_batch_run(states, 0.0, 1e30, 3)
    assert st == [af.AF_OK, af.AF_OK] and n == [3, 3]
    for (g, f, kw), U, ti in zip(insts, states, t):
        cfg = O.make_cfg(g, **kw)
        ref = W.make_state(g, f, GAMMA)
        sto, no, to = O.run(cfg, ref, 0.0, 1e30, 3)
        assert sto == 0 and no == 3
        assert ti == pytest.approx(to, rel=1e-13)
        assert_close(g, U.cpu().numpy(), ref, what="batch vs oracle")


def test_batch_stops_at_t_final_and_counts_attempts():
    insts = instances()[:2]
    solvers = [af.Solver(g, **kw) for g, f, kw in insts]
    states = [S.to_device(W.make_state(g, f, GAMMA)) for S, (g, f, kw) in zip(solvers, insts)]
    t_final = 2e-4
    st, n, t, att = af.Batch(solvers).af_batch_run(states, 0.0, t_final, 10 ** 6)
    assert st == [af.AF_OK, af.AF_OK]
    assert all(abs(ti - t_final) <= 1e-15 * t_final for ti in t)
    assert all(a >= k for a, k in zip(att, n))
    for (g, f, kw), U, ni, ti in zip(insts, states, n, t):
        S = af.Solver(g, **kw)
        V = S.to_device(W.make_state(g, f, GAMMA))
        st1, n1, t1 = S.af_run(V, 0.0, t_final, 10 ** 6, check_every=1)
        assert n1 == ni and t1 == ti
        assert np.array_equal(U.cpu().numpy(), V.cpu().numpy())


def run_batch(insts, precision, steps, variant=None, use_graph=True, aps=4):
    solvers = [af.Solver(g, precision=precision, **kw) for g, f, kw in insts]
    states = [S.to_device(W.make_state(g, f, kw.get("gamma", GAMMA)))
              for S, (g, f, kw) in zip(solvers, insts)]
    B = af.Batch(solvers)
    if variant is not None:
        B.variant = variant
    st, n, t, att = B.af_batch_run(states, 0.0, 1e30, steps, attempts_per_slot=aps,
                                   use_graph=use_graph)
    assert st == [af.AF_OK] * len(insts)
    assert n == [steps] * len(insts)
    return [U.cpu().numpy() for U in states], t, att


@pytest.mark.parametrize("precision", [af.PREC_FP64, af.PREC_MIXED])
def test_every_stage_variant_gives_the_same_result(precision):
    """the tile shapes differ only in how the grid is cut: every site is
    computed by the same arithmetic, so all variants agree to the last bit
    (the instances include grids whose sides are no multiple of any tile)"""
    variants = [i for i, (name, p, ty) in enumerate(af.stage_variants()) if p == precision]
    assert len(variants) >= 2
    insts = instances()
    base = run_batch(insts, precision, 4, variant=variants[0])
    for v in variants[1:]:
        got = run_batch(insts, precision, 4, variant=v)
        assert got[1] == base[1] and got[2] == base[2], af.stage_variants()[v]
        for a, b in zip(got[0], base[0]):
            assert np.array_equal(a, b), af.stage_variants()[v]


def test_set_variant_rejects_the_other_precision():
    g, f, kw = instances()[1]
    B = af.Batch([af.Solver(g, **kw)])
    names = af.stage_variants()
    other = [i for i, (name, p, ty) in enumerate(names) if p != af.PREC_FP64]
    assert names[B.variant][1] == af.PREC_FP64
    with pytest.raises(af.AFError):
        B.variant = other[0]
    with pytest.raises(af.AFError):
        B.variant = len(names)


@pytest.mark.parametrize("precision", [af.PREC_FP64, af.PREC_MIXED])
def test_tune_keeps_the_fastest_variant_and_leaves_the_states_alone(precision):
    insts = W.shock_tube_sweep(5, seed=3, n1_choices=(48, 64, 96, 128))
    solvers = [af.Solver(g, precision=precision, **kw) for g, f, kw in insts]
    states = [S.to_device(W.make_state(g, f, kw["gamma"])) for S, (g, f, kw) in zip(solvers, insts)]
    before = [U.clone() for U in states]
    B = af.Batch(solvers)
    us = B.af_batch_tune(states, 0.0, 1e30, reps=2)
    names = af.stage_variants()
    assert len(us) == len(names)
    for u, (name, p, ty) in zip(us, names):
        assert (u > 0.0) if p == precision else (u == -1.0), (name, u)
    assert names[B.variant][1] == precision
    assert us[B.variant] == min(u for u in us if u > 0.0)
    for a, b in zip(before, states):
        assert torch.equal(a, b)
    # later runs use the chosen variant and still reproduce single runs
    st, n, t, att = B.af_batch_run(states, 0.0, 1e30, 3, use_graph=True)
    assert st == [af.AF_OK] * len(insts) and n == [3] * len(insts)
    for (g, f, kw), U, ti in zip(insts, states, t):
        ref, tr = run_single(g, f, kw, 3, precision)
        assert ti == tr
        assert np.array_equal(U.cpu().numpy(), ref)


def test_sweep_instances_match_the_oracle():
    """two small instances of the randomised shock-tube sweep, FP64, against
    the oracle (random Reynolds numbers and density ratios)"""
    insts = W.shock_tube_sweep(2, seed=11, n1_choices=(24, 40))
    got, t, att = run_batch(insts, af.PREC_FP64, 3)
    for (g, f, kw), U, ti in zip(insts, got, t):
        cfg = O.make_cfg(g, **kw)
        ref = W.make_state(g, f, kw["gamma"])
        sto, no, to = O.run(cfg, ref, 0.0, 1e30, 3)
        assert sto == 0 and no == 3
        assert ti == pytest.approx(to, rel=1e-13)
        assert_close(g, U, ref, what="sweep instance vs oracle")
