"""GPU checks of 1D Dirichlet sides on the paper's viscous-shock accuracy
test (Sec. 4, Becker's exact solution): the GPU's steps against the
oracle's (FP64 parity bar, growing with the steps compared), with and
without limiting, SSP-RK54 and SSP-RK3; and the GPU's own fourth-order
convergence to the exact solution."""
import numpy as np
import pytest

import oracle as O
from parity import assert_close
from paper_2609_29081_amd import af
from paper_2609_29081_amd import workloads as W

pytestmark = pytest.mark.gpu

GAMMA = 1.4


def setup(n, M0, mu, limiter, rk):
    g, prim, bcs = W.becker_shock_1d(n, M0=M0, mu=mu)
    U = W.make_state(g, lambda x: prim(x, 0.0), GAMMA, nq=40)
    cfl = dict(cfl_c=1.04, cfl_v=0.33) if rk == 54 else dict(cfl_c=0.2, cfl_v=0.15)
    kw = dict(mu=mu, Pr=0.75, limiter=limiter, rk=rk, **cfl)
    cfg = O.make_cfg(g, gamma=GAMMA, bcstate=bcs, **kw)
    S = af.Solver(g, gamma=GAMMA, bcstate=bcs, **kw)
    return g, prim, U, cfg, S


@pytest.mark.parametrize("n,M0,mu,limiter,rk", [(80, 3.0, 1e-2, 0, 54),
                                                (160, 20.0, 1e-3, af.LIM_ALL, 54),
                                                (120, 20.0, 1e-3, af.LIM_ALL, 3)])
def test_dirichlet_steps_match_the_oracle(n, M0, mu, limiter, rk):
    g, prim, U, cfg, S = setup(n, M0, mu, limiter, rk)
    Ud = S.to_device(U)
    st, ns, t = O.run(cfg, U, 0.0, 1e30, 12)
    stg, nsg, tg = S.af_run(Ud, 0.0, 1e30, 12, check_every=4)
    assert st == 0 and stg == af.AF_OK and ns == nsg == 12
    assert tg == pytest.approx(t, rel=1e-12)
    assert_close(g, Ud.cpu().numpy(), U, tol=1e-11, what=f"Becker M0={M0} rk={rk}")


def test_gpu_reaches_fourth_order_on_the_exact_solution():
    errs = []
    for n in (320, 640):
        g, prim, U, cfg, S = setup(n, 3.0, 1e-2, 0, 54)
        Ud = S.to_device(U)
        st, ns, t = S.af_run(Ud, 0.0, 0.2, 10 ** 6, check_every=16)
        assert st == af.AF_OK and t == pytest.approx(0.2, rel=1e-14)
        ref = W.make_state(g, lambda x: prim(x, 0.2), GAMMA, nq=40)
        r = g.split(Ud.cpu().numpy())["avg"][0]
        errs.append(float(np.abs(r - g.split(ref)["avg"][0]).sum() * g.dx))
    assert np.log2(errs[0] / errs[1]) > 3.6, errs


def test_dirichlet_is_one_dimensional():
    g, f = W.random_smooth_2d(8, 8, seed=0, amp=0.1)
    S = af.Solver(g)
    with pytest.raises(af.AFError):
        af._check(af.lib().af_set_bc(S.ctx, 0, af.DIRICHLET))
