"""GPU steps with a source term (af_step_source) on the paper's manufactured
Taylor-Green vortex (Sec. 4): against the oracle's steps with the same
source states (FP64 parity bar), and the GPU's own fourth-order
convergence to the prescribed solution."""
import numpy as np
import pytest
import torch

import oracle as O
from parity import assert_close
from paper_2609_29081_amd import af
from paper_2609_29081_amd import workloads as W

pytestmark = pytest.mark.gpu

GAMMA = 1.4
KW = dict(mu=1e-5, Pr=1.0, cfl_c=0.52, cfl_v=0.165)


@pytest.mark.parametrize("rk", [3, 54])
def test_source_steps_match_the_oracle(rk):
    g, prim, src = W.taylor_green_2d(16)
    U = W.make_state(g, lambda x, y: prim(x, y, 0.0), GAMMA)
    cfg = O.make_cfg(g, gamma=GAMMA, rk=rk, **KW)
    S = af.Solver(g, gamma=GAMMA, rk=rk, **KW)
    Ud = S.to_device(U)
    dt = 0.5 * O.dt(cfg, U)
    c = af.stage_times(rk)
    assert c == pytest.approx(O.stage_times(rk), rel=1e-15)
    for k in range(3):
        srcs = [src(k * dt + ck * dt) for ck in c]
        U, fl = O.step_source(cfg, U, dt, srcs)
        st = S.af_step_source(Ud, dt, [S.to_device(x) for x in srcs])
        assert fl == 0 and st == af.AF_OK
        assert_close(g, Ud.cpu().numpy(), U, tol=1e-12 * (k + 1), what=f"rk{rk} step {k}")


def test_gpu_taylor_green_is_fourth_order():
    errs = []
    for n in (32, 64):
        g, prim, src = W.taylor_green_2d(n)
        U = W.make_state(g, lambda x, y: prim(x, y, 0.0), GAMMA)
        cfg = O.make_cfg(g, gamma=GAMMA, rk=54, **KW)
        S = af.Solver(g, gamma=GAMMA, rk=54, **KW)
        Ud = S.to_device(U)
        T = 0.2
        ns = int(np.ceil(T / O.dt(cfg, U)))
        dt = T / ns
        c = af.stage_times(54)
        for k in range(ns):
            st = S.af_step_source(Ud, dt, [S.to_device(src(k * dt + ck * dt)) for ck in c])
            assert st == af.AF_OK
        ref = W.make_state(g, lambda x, y: prim(x, y, T), GAMMA)
        errs.append(float(np.abs(Ud.cpu().numpy() - ref).mean()))
    assert np.log2(errs[0] / errs[1]) > 3.5, errs
