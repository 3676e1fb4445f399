"""Pins of the oracle's learned-blend pieces (CPU): the reference network
(gradient against finite differences, Adam's first step in closed form,
bfloat16 rounding on exact ties, the rounded inference reducing to the FP64
forward pass when nothing rounds), the face features (their definition on
an interior face, invariance under a uniform velocity, the symmetry between
x- and y-faces under transposition, zero on a constant state) and the
blend-mode stage (theta_nn = 1 is the stage without the smoothness blend,
theta_nn = 0 gives the low-order cell fluxes, every theta_nn in [0, 1]
conserves mass and keeps admissible averages admissible)."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
from paper_2609_29081_amd import workloads as W

GAMMA = 1.4


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    params = W.mlp_init(3).astype(np.float64)
    params += rng.normal(0.0, 0.05, size=params.shape)  # nonzero biases too
    X = rng.normal(0.0, 1.0, size=(13, M.NIN))
    y = rng.uniform(0.0, 1.0, size=13)
    loss, g = M.loss_and_grad(params, X, y)
    idx = np.concatenate([rng.choice(M.NPARAM, 60, replace=False), [M.NPARAM - 1]])
    h = 1e-6
    for q in idx:
        e = np.zeros(M.NPARAM)
        e[q] = h
        lp, _ = M.loss_and_grad(params + e, X, y)
        lm, _ = M.loss_and_grad(params - e, X, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[q]) <= 1e-7 * max(1.0, abs(fd)), (q, fd, g[q])


def test_adam_first_step_moves_each_parameter_by_lr_against_its_gradient_sign():
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    p1, m, v = M.adam(p0, g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=0.0)
    assert np.allclose(p1, p0 - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounds_to_nearest_even():
    one = 1.0
    assert M.bf16(one) == 1.0
    assert M.bf16(1.0 + 2.0 ** -8) == 1.0                  # tie: even mantissa 0
    assert M.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie: even mantissa 2
    assert M.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7  # above the tie
    assert M.bf16(-2.5) == -2.5


def test_rounded_inference_is_the_forward_pass_when_nothing_rounds():
    rng = np.random.default_rng(2)
    P = M.unpack(W.mlp_init(5).astype(np.float64))
    # weights and inputs exactly representable in bfloat16, tiny weights in
    # the second layer so that h1 need not be representable
    P["W1"] = M.bf16(P["W1"])
    P["W2"] = np.zeros_like(P["W2"])
    P["w3"] = M.bf16(P["w3"])
    P["b2"] = M.bf16(rng.uniform(-0.5, 0.5, size=M.NH)).astype(np.float32).astype(np.float64)
    params = M.pack(P)
    X = M.bf16(rng.normal(0.0, 1.0, size=(9, M.NIN)))
    z, _ = M.forward(params, X)
    assert np.allclose(M.infer_bf16(params, X), np.clip(z, 0.0, 1.0), rtol=0, atol=1e-15)


def smooth_state(n1, n2, seed, bc=(W.PERIODIC,) * 4):
    g, f = W.random_smooth_2d(n1, n2, seed=seed, bc=bc, amp=0.15)
    return g, W.make_state(g, f, GAMMA)


def prims_of_averages(g, U):
    P = g.split(U)["avg"]
    r = P[0]
    u, v = P[1] / r, P[2] / r
    p = (GAMMA - 1.0) * (P[3] - 0.5 * r * (u * u + v * v))
    return r, u, v, p


def test_features_follow_their_definition_on_interior_faces():
    g, U = smooth_state(9, 8, 4)
    cfg = O.make_cfg(g, gamma=GAMMA)
    F = O.blend_features(cfg, U)
    r, u, v, p = prims_of_averages(g, U)   # arrays [j, i]
    n1, n2 = g.n1, g.n2
    nfx = n2 * (n1 + 1)
    for d, (i, j) in [(0, (4, 3)), (0, (3, 5)), (1, (4, 3)), (1, (5, 4))]:
        rows = []
        if d == 0:   # face between cells (i-1, j) and (i, j); n = x, t = y
            cell = lambda m, s: (j + s, i + (m if m < 0 else m - 1))
            un, ut = u, v
            f = j * (n1 + 1) + i
        else:        # face between (i, j-1) and (i, j); n = y, t = x
            cell = lambda m, s: (j + (m if m < 0 else m - 1), i + s)
            un, ut = v, u
            f = nfx + j * n1 + i
        a, b = cell(-1, 0), cell(1, 0)
        rf, pf = (r[a] + r[b]) / 2, (p[a] + p[b]) / 2
        unf, utf = (un[a] + un[b]) / 2, (ut[a] + ut[b]) / 2
        cf = np.sqrt(GAMMA * pf / rf)
        for s in (-1, 0, 1):
            for m in (-2, -1, 1, 2):
                q = cell(m, s)
                rows += [np.log(p[q] / pf), (un[q] - unf) / cf, (ut[q] - utf) / cf]
        rows += [np.log(r[cell(m, 0)] / rf) for m in (-2, -1, 1, 2)]
        assert np.allclose(F[f], rows, rtol=1e-13, atol=1e-14), (d, i, j)


def test_features_are_zero_on_a_constant_state_and_ignore_a_uniform_velocity():
    g, f = W.shock_tube_2d(10, 6, rho_left=7.0)
    cfg = O.make_cfg(g, gamma=GAMMA)
    gc, fc = W.random_smooth_2d(8, 7, seed=0, amp=0.0)
    Uc = W.make_state(gc, fc, GAMMA)
    assert np.abs(O.blend_features(O.make_cfg(gc, gamma=GAMMA), Uc)).max() < 1e-13
    # periodic smooth field, then the same field carried by a uniform velocity
    g2, U2 = smooth_state(8, 7, 9)
    cfg2 = O.make_cfg(g2, gamma=GAMMA)
    P = g2.split(U2)
    V = U2.copy()
    Q = g2.split(V)
    for name in P:
        r = P[name][0]
        e_int = P[name][3] - 0.5 * (P[name][1] ** 2 + P[name][2] ** 2) / r
        Q[name][1][...] = P[name][1] + 0.7 * r
        Q[name][2][...] = P[name][2] - 0.4 * r
        Q[name][3][...] = e_int + 0.5 * (Q[name][1] ** 2 + Q[name][2] ** 2) / r
    assert np.allclose(O.blend_features(cfg2, V), O.blend_features(cfg2, U2), rtol=0, atol=1e-11)


def transpose_state(g, U):
    """the state of the transposed problem (x <-> y, momenta swapped)"""
    gt = W.Grid(dim=2, n1=g.n2, n2=g.n1, x0=g.y0, x1=g.y1, y0=g.x0, y1=g.x1,
                bc=(g.bc[2], g.bc[3], g.bc[0], g.bc[1]))
    P = g.split(U)
    out = np.empty_like(U)
    Q = gt.split(out)
    for a, b in (("avg", "avg"), ("xe", "ye"), ("ye", "xe"), ("co", "co")):
        for k, kk in ((0, 0), (1, 2), (2, 1), (3, 3)):
            Q[b][kk][...] = P[a][k].T
    return gt, out


def test_x_faces_and_y_faces_agree_under_transposition():
    g, f = W.random_smooth_2d(7, 5, seed=6, bc=(W.NOSLIP, W.OUTFLOW, W.SYMMETRY, W.NOSLIP),
                              amp=0.15)
    U = W.make_state(g, f, GAMMA)
    gt, Ut = transpose_state(g, U)
    F = O.blend_features(O.make_cfg(g, gamma=GAMMA), U)
    Ft = O.blend_features(O.make_cfg(gt, gamma=GAMMA), Ut)
    n1, n2 = g.n1, g.n2
    nfx = n2 * (n1 + 1)
    # x-face (i, j) of the original is y-face (j, i) of the transposed grid
    fx = F[:nfx].reshape(n2, n1 + 1, 40)
    fy_t = Ft[gt.n2 * (gt.n1 + 1):].reshape(gt.n2 + 1, gt.n1, 40)
    assert np.allclose(fx, np.transpose(fy_t, (1, 0, 2)), rtol=1e-12, atol=1e-13)


def test_blend_one_is_the_stage_without_the_smoothness_blend():
    g, f = W.shock_tube_2d(16, 10, rho_left=30.0)
    U = W.make_state(g, f, GAMMA)
    cfg_all = O.make_cfg(g, gamma=GAMMA, mu=0.005, Pr=0.73)
    cfg_nos = O.make_cfg(g, gamma=GAMMA, mu=0.005, Pr=0.73,
                         limiter=O.LIM_PP | O.LIM_POINT | O.LIM_CENTRE)
    dt = 0.5 * O.dt(cfg_all, U)
    a, fa = O.fe_blend(cfg_all, U, dt, np.ones(O.nfaces(cfg_all)))
    b, fb = O.fe(cfg_nos, U, dt)
    assert fa == fb and np.array_equal(a, b)


def test_blend_zero_gives_the_low_order_cell_fluxes():
    g, f = W.shock_tube_2d(16, 10, rho_left=30.0)
    U = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, gamma=GAMMA, mu=0.005, Pr=0.73)
    cfg_lo = O.make_cfg(g, gamma=GAMMA, mu=0.005, Pr=0.73, limiter=O.LIM_ALL | O.LIM_LOWONLY)
    dt = 0.5 * O.dt(cfg, U)
    a, _ = O.fe_blend(cfg, U, dt, np.zeros(O.nfaces(cfg)))
    lo, _ = O.fe(cfg_lo, U, dt)
    plain, _ = O.fe(cfg, U, dt)
    na = 4 * g.n1 * g.n2
    assert np.array_equal(a[:na], lo[:na])          # cell averages: low order
    assert np.array_equal(a[na:], plain[na:])       # point values: untouched


@pytest.mark.parametrize("seed", [0, 1])
def test_any_blend_conserves_and_keeps_averages_admissible(seed):
    th_of = lambda cfg: np.random.default_rng(seed).uniform(0.0, 1.0, size=O.nfaces(cfg))
    # conservation: periodic field, every component's sum of averages
    g, U = smooth_state(12, 10, 3 + seed)
    cfg = O.make_cfg(g, gamma=GAMMA, mu=1e-3)
    out, fl = O.fe_blend(cfg, U, O.dt(cfg, U), th_of(cfg))
    P0, P1 = g.split(U)["avg"], g.split(out)["avg"]
    for k in range(4):
        assert abs(P1[k].sum() - P0[k].sum()) <= 1e-13 * np.abs(P0[k]).sum()
    # admissibility: a near-vacuum centre that the limiter must act on
    g, f = W.double_rarefaction(20, 12, speed=1.8, angle=0.0)
    U = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, gamma=GAMMA, mu=1e-3)
    out, fl = O.fe_blend(cfg, U, O.dt(cfg, U), th_of(cfg))
    assert fl & O.FLAG_CELL_LOW == 0
    P1 = g.split(out)["avg"]
    r = P1[0]
    p = (GAMMA - 1.0) * (P1[3] - 0.5 * (P1[1] ** 2 + P1[2] ** 2) / r)
    assert r.min() > 0.0 and p.min() > 0.0


def test_blend_equal_to_theta_s_is_the_plain_stage():
    g, f = W.shock_tube_2d(18, 12, rho_left=40.0)
    U = W.make_state(g, f, GAMMA)
    cfg = O.make_cfg(g, gamma=GAMMA, mu=0.005, Pr=0.73)
    for _ in range(4):  # the gas at rest has no compression yet
        assert O.step(cfg, U)[0] == 0
    dt = 0.5 * O.dt(cfg, U)
    plain, fl, ts, _ = O.fe(cfg, U, dt, want_theta=True)
    assert (ts < 0.999).any()  # the smoothness blend acts somewhere
    out, fb = O.fe_blend(cfg, U, dt, ts)
    assert fb == fl and np.array_equal(out, plain)
