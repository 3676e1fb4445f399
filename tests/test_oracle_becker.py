"""The paper's 1D accuracy test (Sec. 4, the moving viscous shock with
Becker's exact solution for Pr = 3/4) as a pin of the oracle: Dirichlet
sides holding the far-field states, SSP-RK54 with C^c = 1.04 and
C^v = 0.33, t = 0.2.  Without limiting (M0 = 3, mu = 1e-2) the L1 error of
the density averages against the exact averages falls at fourth order, as
the paper reports; with all limiters (M0 = 20, mu = 1e-3) the run stays
admissible and its error falls too."""
import numpy as np
import pytest

import oracle as O
from paper_2609_29081_amd import workloads as W

GAMMA = 1.4


def exact_state(g, prim, t):
    return W.make_state(g, lambda x: prim(x, t), GAMMA, nq=40)


def l1_error(n, M0, mu, limiter, t_final=0.2):
    g, prim, bcs = W.becker_shock_1d(n, M0=M0, mu=mu)
    U = exact_state(g, prim, 0.0)
    cfg = O.make_cfg(g, gamma=GAMMA, mu=mu, Pr=0.75, limiter=limiter, rk=54, cfl_c=1.04,
                     cfl_v=0.33, bcstate=bcs)
    st, ns, t = O.run(cfg, U, 0.0, t_final)
    assert st == 0 and t == pytest.approx(t_final, rel=1e-14)
    ref = exact_state(g, prim, t_final)
    r, rr = g.split(U)["avg"][0], g.split(ref)["avg"][0]
    return float(np.abs(r - rr).sum() * g.dx), U, g


def test_fourth_order_without_limiting():
    # measured: 1.2e-2 .. 5.4e-6 over N = 40 .. 640, rates 1.2, 3.3, 3.2, 3.8
    # (the shock, about 0.016 wide, is resolved from N ~ 160 on)
    errs = [l1_error(n, 3.0, 1e-2, 0)[0] for n in (320, 640)]
    rate = np.log2(errs[0] / errs[1])
    assert rate > 3.6, (errs, rate)


def test_limited_strong_shock_stays_admissible_and_converges():
    # mu = 1e-3 makes the shock about 0.0016 wide: at these grids it is
    # captured over a cell or two, so the error falls at first order here
    e1, U, g = l1_error(640, 20.0, 1e-3, O.LIM_ALL)
    e2, _, _ = l1_error(1280, 20.0, 1e-3, O.LIM_ALL)
    P = g.split(U)
    for name in P:
        r = P[name][0]
        p = (GAMMA - 1.0) * (P[name][2] - 0.5 * P[name][1] ** 2 / r)
        assert r.min() > 0 and p.min() > 0
    assert e2 < 0.5 * e1, (e1, e2)
