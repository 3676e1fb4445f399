"""GPU checks of the learned blend coefficient against the oracle.

* Features: the GPU computes them in FP32 from the FP64 averages; the
  oracle in FP64.  Each is a logarithm or a velocity difference over a sound
  speed, a few FP32 operations, so the bar is 1e-5 absolute plus 1e-5
  relative.
* Blend-mode stage with a given blend array (seeded random coefficients in
  [0, 1]): the FP64 stage to the FP64 parity bar, the mixed stage to its own
  bar; flags exactly.
* theta^s written out by a plain stage (the training targets): FP64 parity.
* Inference: both sides round the weights and the layer inputs to bfloat16.
  The GPU's FP32 features and hidden values can round to a neighbouring
  bfloat16 value where the oracle's FP64 ones round the other way (a
  relative change of 2^-8 in one input), and the sums run in FP32 against
  FP64; the bar is 1e-2 on every face and 1e-3 on 99 % of them.
* Training: the FP32 gradient against the FP64 one on the same rows, to
  1e-4 of the largest gradient entry; one Adam step to 1e-6 relative; and a
  few hundred steps lower the loss on the method's own theta^s.
* AF_LIM_LEARNED steps: admissible, conservative, and close to the oracle's
  learned step (whose blend comes from the oracle's own features and
  network)."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import mlp as M
from parity import assert_close, REL_TOL_FP64
from paper_2609_29081_amd import af
from paper_2609_29081_amd import workloads as W

pytestmark = pytest.mark.gpu

GAMMA = 1.4
REL_TOL_MIXED = 1e-5


def cases():
    out = []
    g, f = W.shock_tube_2d(37, 21, rho_left=60.0)
    out.append(("shock_tube", g, W.make_state(g, f, GAMMA), dict(mu=0.005, Pr=0.73)))
    g, f = W.random_smooth_2d(20, 17, seed=2, amp=0.15)
    out.append(("periodic", g, W.make_state(g, f, GAMMA), dict(mu=1e-3, Pr=0.72)))
    g, f = W.random_smooth_2d(19, 23, seed=7, bc=(W.NOSLIP, W.OUTFLOW, W.SYMMETRY, W.NOSLIP),
                              amp=0.15)
    out.append(("mixed_walls", g, W.make_state(g, f, GAMMA), dict(mu=0.01, Pr=0.72)))
    return out


@pytest.mark.parametrize("case", cases(), ids=lambda c: c[0])
def test_features_match_the_oracle(case):
    name, g, U, kw = case
    S = af.Solver(g, **kw)
    got = S.af_blend_features(S.to_device(U)).cpu().numpy().astype(np.float64)
    ref = O.blend_features(O.make_cfg(g, gamma=GAMMA, **kw), U)
    assert got.shape == ref.shape
    err = np.abs(got - ref) - 1e-5 * np.abs(ref)
    assert err.max() <= 1e-5, (name, float(np.abs(got - ref).max()))


def stage_pair(g, U, kw, theta, precision, k, dt_scale=0.5):
    cfg = O.make_cfg(g, gamma=GAMMA, **kw)
    dt = dt_scale * O.dt(cfg, U)
    S = af.Solver(g, precision=precision, **kw)
    Ud = S.to_device(U)
    fe, fl = O.fe_blend(cfg, U, dt, theta)
    Uk = U if k == 0 else fe  # stage k from the same input twice
    if k == 0:
        ref = fe
        Un_d = None
    else:
        fe2, fl = O.fe_blend(cfg, Uk, dt, theta)
        a, b = (0.75, 0.25) if k == 1 else (1.0 / 3.0, 2.0 / 3.0)
        ref = a * U + b * fe2
        Un_d = Ud
    out = torch.empty_like(Ud)
    S.af_reset_flags()
    th = torch.as_tensor(theta, dtype=torch.float32, device=S.device)
    S.af_rk_stage_blend(k, Un_d, S.to_device(Uk), out, dt=dt, theta=th)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref, S.af_read_flags(), fl


@pytest.mark.parametrize("case", cases(), ids=lambda c: c[0])
@pytest.mark.parametrize("k", [0, 1, 2])
def test_blend_stage_matches_the_oracle_fp64(case, k):
    name, g, U, kw = case
    # coefficients exactly representable in FP32, so both sides use the same
    theta = np.random.default_rng(k).uniform(0.0, 1.0, size=g.n2 * (g.n1 + 1) + (g.n2 + 1) * g.n1)
    theta = theta.astype(np.float32).astype(np.float64)
    got, ref, fl, fl_ref = stage_pair(g, U, kw, theta, af.PREC_FP64, k)
    assert fl == fl_ref
    assert_close(g, got, ref, tol=REL_TOL_FP64, what=f"{name} stage {k}")


@pytest.mark.parametrize("case", cases()[:2], ids=lambda c: c[0])
def test_blend_stage_matches_the_oracle_mixed(case):
    name, g, U, kw = case
    theta = np.random.default_rng(5).uniform(0.0, 1.0, size=g.n2 * (g.n1 + 1) + (g.n2 + 1) * g.n1)
    theta = theta.astype(np.float32).astype(np.float64)
    got, ref, fl, fl_ref = stage_pair(g, U, kw, theta, af.PREC_MIXED, 0)
    assert fl == fl_ref
    assert_close(g, got, ref, tol=REL_TOL_MIXED, what=f"{name} mixed")


@pytest.mark.parametrize("case", cases(), ids=lambda c: c[0])
def test_theta_s_written_by_a_plain_stage(case):
    name, g, U, kw = case
    cfg = O.make_cfg(g, gamma=GAMMA, **kw)
    dt = 0.5 * O.dt(cfg, U)
    _, _, ts_ref, _ = O.fe(cfg, U, dt, want_theta=True)
    S = af.Solver(g, **kw)
    Ud = S.to_device(U)
    out = torch.empty_like(Ud)
    ts = torch.full((S.face_count,), -1.0, dtype=torch.float32, device=S.device)
    S.af_rk_stage_blend(0, None, Ud, out, dt=dt, theta_s_out=ts)
    got = ts.cpu().numpy().astype(np.float64)
    assert np.abs(got - ts_ref).max() <= 1e-6  # FP32 storage of an FP64 value
    assert (got >= 0).all() and (got <= 1).all()


def trained_like_params(seed):
    """initial weights with nonzero biases (a network away from its start)"""
    p = W.mlp_init(seed).astype(np.float64)
    p += np.random.default_rng(seed + 100).normal(0.0, 0.05, size=p.shape)
    return p.astype(np.float32)


@pytest.mark.parametrize("case", cases(), ids=lambda c: c[0])
def test_inference_matches_the_oracle(case):
    name, g, U, kw = case
    params = trained_like_params(3)
    S = af.Solver(g, **kw)
    P = torch.as_tensor(params, device=S.device)
    S.af_set_blend_net(P)
    got = S.af_blend_infer(S.to_device(U)).cpu().numpy().astype(np.float64)
    X = O.blend_features(O.make_cfg(g, gamma=GAMMA, **kw), U)
    ref = M.infer_bf16(params.astype(np.float64), X)
    # periodic duplicates: the stage reads the first face of a line only
    d = np.abs(got - ref)
    assert d.max() <= 1e-2, (name, float(d.max()))
    assert np.quantile(d, 0.99) <= 1e-3, (name, float(np.quantile(d, 0.99)))


def oracle_rows(n_rows=3000, seed=0):
    """features and theta^s of a few shock-tube stages, from the oracle"""
    g, f = W.shock_tube_2d(48, 24, rho_left=80.0)
    U = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, gamma=GAMMA, mu=0.004, Pr=0.73)
    Xs, ys = [], []
    for _ in range(3):
        X = O.blend_features(cfg, U)
        dt = O.dt(cfg, U)
        _, _, ts, _ = O.fe(cfg, U, 0.5 * dt, want_theta=True)
        Xs.append(X)
        ys.append(ts)
        st, _, _, _ = O.step(cfg, U)
        assert st == 0
    X, y = np.concatenate(Xs), np.concatenate(ys)
    idx = np.random.default_rng(seed).permutation(len(y))[:n_rows]
    return X[idx].astype(np.float32), y[idx].astype(np.float32)


def test_gradient_matches_the_oracle():
    X, y = oracle_rows(1000)
    params = trained_like_params(4)
    dev = torch.device("cuda:0")
    grad, loss = af.mlp_grad(torch.as_tensor(X, device=dev), torch.as_tensor(y, device=dev),
                             torch.as_tensor(params, device=dev))
    torch.cuda.synchronize()
    lref, gref = M.loss_and_grad(params.astype(np.float64), X.astype(np.float64),
                                 y.astype(np.float64))
    g = grad.cpu().numpy().astype(np.float64)
    assert np.abs(g - gref).max() <= 1e-4 * np.abs(gref).max()
    assert abs(float(loss.item()) - lref) <= 1e-5 * max(lref, 1e-12)


def test_adam_step_matches_the_oracle():
    rng = np.random.default_rng(9)
    p = rng.normal(size=M.NPARAM).astype(np.float32)
    g = rng.normal(size=M.NPARAM).astype(np.float32)
    m = (0.1 * rng.normal(size=M.NPARAM)).astype(np.float32)
    v = (0.01 * rng.uniform(size=M.NPARAM)).astype(np.float32)
    dev = torch.device("cuda:0")
    P, G, Mm, V = (torch.as_tensor(a, device=dev).clone() for a in (p, g, m, v))
    af.mlp_adam(P, G, Mm, V, 7, 1e-3)
    pr, mr, vr = M.adam(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                        v.astype(np.float64), 7, 1e-3)
    # FP32 state: the bar is a few FP32 roundings of the parameter and of
    # the update
    upd = np.abs(pr - p.astype(np.float64))
    assert (np.abs(P.cpu().numpy() - pr) <= 4e-7 * (np.abs(pr) + upd) + 1e-9).all()
    assert np.allclose(Mm.cpu().numpy(), mr, rtol=1e-6, atol=1e-7)
    assert np.allclose(V.cpu().numpy(), vr, rtol=1e-6, atol=1e-9)


def test_training_lowers_the_loss_on_the_methods_theta_s():
    X, y = oracle_rows(3000, seed=1)
    dev = torch.device("cuda:0")
    Xd, yd = torch.as_tensor(X, device=dev), torch.as_tensor(y, device=dev)
    P = torch.as_tensor(W.mlp_init(0), device=dev).clone()
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    _, l0 = af.mlp_grad(Xd, yd, P)
    af.mlp_train(Xd, yd, P, m, v, 0, 300, 256, 3e-3)
    _, l1 = af.mlp_grad(Xd, yd, P)
    torch.cuda.synchronize()
    assert float(l1.item()) < 0.3 * float(l0.item()), (float(l0.item()), float(l1.item()))


def oracle_learned_step(cfg, U, params, dt):
    """one SSP-RK3 step whose stages take their blend from the oracle's own
    features and network (no halving: dt is small)"""
    def fe(V):
        th = M.infer_bf16(params, O.blend_features(cfg, V))
        out, fl = O.fe_blend(cfg, V, dt, th)
        assert fl == 0
        return out
    U1 = fe(U)
    U2 = 0.75 * U + 0.25 * fe(U1)
    return U / 3.0 + 2.0 / 3.0 * fe(U2)


def test_learned_steps_are_admissible_conservative_and_near_the_oracle():
    g, f = W.random_smooth_2d(24, 20, seed=4, amp=0.2)
    U = W.make_state(g, f, GAMMA)
    kw = dict(mu=1e-3, Pr=0.72)
    params = trained_like_params(6)
    S = af.Solver(g, limiter=af.LIM_ALL | af.LIM_LEARNED, **kw)
    S.af_set_blend_net(torch.as_tensor(params, device=S.device))
    cfg = O.make_cfg(g, gamma=GAMMA, **kw)
    dt = 0.5 * O.dt(cfg, U)
    Ud = S.to_device(U)
    st, dtu, h = S.af_step(Ud, dt=dt)
    assert st == af.AF_OK and h == 0
    got = Ud.cpu().numpy()
    ref = oracle_learned_step(cfg, U, params.astype(np.float64), dt)
    assert S.af_check_admissible(Ud) == 0
    P0, P1 = g.split(U)["avg"], g.split(got)["avg"]
    for k in range(4):
        assert abs(P1[k].sum() - P0[k].sum()) <= 1e-12 * np.abs(P0[k]).sum()
    # blends differ only where a bfloat16 rounding went the other way
    assert_close(g, got, ref, tol=1e-4, what="learned step vs oracle")


def test_learned_limiter_needs_a_network():
    g, f = W.random_smooth_2d(8, 8, seed=1, amp=0.1)
    S = af.Solver(g, limiter=af.LIM_ALL | af.LIM_LEARNED)
    Ud = S.to_device(W.make_state(g, f, GAMMA))
    with pytest.raises(af.AFError):
        S.af_step(Ud, dt=1e-4)


def test_training_brings_learned_runs_to_the_plain_limiter():
    """what the trained network gains: trained on the plain limiter's theta^s
    of one run, its learned-blend run ends much nearer the plain run than
    the untrained network's or a run without any smoothness blend"""
    g, f = W.shock_tube_2d(160, 80, rho_left=120.0)
    U0 = W.make_state(g, f, GAMMA)
    kw = dict(mu=0.005, Pr=0.73)
    dev = torch.device("cuda:0")
    S = af.Solver(g, **kw)
    U = S.to_device(U0)
    tmp = torch.empty_like(U)
    Xs, ys, done = [], [], 0
    # the first steps, where the diaphragm's jump becomes a viscous shock,
    # are the faces the blend matters most for
    for n in (1, 2, 3, 5, 10, 20):
        st, _, _ = S.af_run(U, 0.0, 1e30, n - done, check_every=1)
        done = n
        assert st == af.AF_OK
        Xs.append(S.af_blend_features(U))
        ts = torch.empty(S.face_count, dtype=torch.float32, device=dev)
        S.af_rk_stage_blend(0, None, U, tmp, dt=0.0, theta_s_out=ts)
        ys.append(ts)
    X, y = torch.cat(Xs), torch.cat(ys)
    P0 = torch.as_tensor(W.mlp_init(0), device=dev)
    P = P0.clone()
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    idx = torch.as_tensor(W.balanced_rows(y.cpu().numpy(), seed=0), device=dev)
    af.mlp_train(X[idx].contiguous(), y[idx].contiguous(), P, m, v, 0, 6000, 512, 2e-3)

    def run(limiter, net, t_final):
        R = af.Solver(g, limiter=limiter, **kw)
        if net is not None:
            R.af_set_blend_net(net)
        V = R.to_device(U0)
        st, n, t = R.af_run(V, 0.0, t_final, 10 ** 6, check_every=1)
        assert st == af.AF_OK
        assert R.af_check_admissible(V) == 0
        return g.split(V.cpu().numpy())["avg"][0], t

    plain, t_end = run(af.LIM_ALL, None, 2.5e-3)
    e = {}
    for name, lim, net in (("trained", af.LIM_ALL | af.LIM_LEARNED, P),
                           ("untrained", af.LIM_ALL | af.LIM_LEARNED, P0),
                           ("no_smoothness", af.LIM_PP | af.LIM_POINT | af.LIM_CENTRE, None)):
        rho, t = run(lim, net, t_end)
        assert t == pytest.approx(t_end, rel=1e-12)
        e[name] = float(np.abs(rho - plain).sum() * g.dx * g.dy)
    assert e["trained"] < 0.5 * e["untrained"], e
    assert e["trained"] < 0.5 * e["no_smoothness"], e
