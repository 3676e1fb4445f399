"""The smooth periodic density wave with a vortex at the sizes of its sweep
(256^2 to 2048^2), launched as af_run launches it on the GPU.

* At 256^2, 512^2 and 1024^2: one RK3 step at the CFL dt in FP64 against
  the FP64 oracle, to the FP64 tolerance, and the same step with FP32
  stencils to the mixed-precision stage's bar.
* At 2048^2, the largest: one RK3 step at the CFL dt (three complete
  stages) against the FP64 oracle, to the FP64 tolerance, and 100 RK3
  steps in FP64 and with FP32 stencils, held to what holds at any
  size: the cell averages' sums (mass, momentum, energy) stay what they
  were to round-off on a periodic grid, every DOF stays admissible, and the
  FP32-stencil run stays within a stated relative L1 distance of the FP64
  run (the oracle would take minutes for 100 steps at this size)."""
import numpy as np
import pytest

import oracle as O
from parity import assert_close
from paper_2609_29081_amd import af
from paper_2609_29081_amd import workloads as W

pytestmark = pytest.mark.gpu

GAMMA = 1.4
N = 2048
KW = dict(mu=1e-3, Pr=0.72)


@pytest.mark.parametrize("n", [256, 512, 1024])
def test_vortex_sweep_sizes_step_against_the_oracle(n):
    g, f = W.vortex_wave_2d(n)
    U0 = W.make_state(g, f, GAMMA)
    U = U0.copy()
    cfg = O.make_cfg(g, **KW)
    st, dtu, h, fl = O.step(cfg, U, 0.0, 0.0)
    assert st == 0 and h == 0
    for prec, tol in ((af.PREC_FP64, 2e-12), (af.PREC_MIXED, 1e-5)):
        S = af.Solver(g, precision=prec, **KW)
        Ud = S.to_device(U0)
        stg, nst, t = S.af_run(Ud, 0.0, 1e30, 1, check_every=1)
        assert stg == af.AF_OK and nst == 1
        assert t == pytest.approx(dtu, rel=1e-12)
        worst = assert_close(g, Ud.cpu().numpy(), U, tol=tol, what=f"vortex {n}^2 precision {prec}")
        print(f"vortex {n}^2, precision {prec}, one step: worst relative error {worst:.3e}")


@pytest.fixture(scope="module")
def vortex():
    """the initial state (its cell averages by 5x5 Gauss-Legendre take most
    of a minute on the host, so both tests share it)"""
    g, f = W.vortex_wave_2d(N)
    return g, W.make_state(g, f, GAMMA)


def test_vortex_2048_step_against_the_oracle(vortex):
    g, U0 = vortex
    U = U0.copy()
    cfg = O.make_cfg(g, **KW)
    S = af.Solver(g, **KW)
    Ud = S.to_device(U)
    st, dtu, h, fl = O.step(cfg, U, 0.0, 0.0)
    assert st == 0 and h == 0
    stg, n, t = S.af_run(Ud, 0.0, 1e30, 1, check_every=1)
    assert stg == af.AF_OK and n == 1
    assert t == pytest.approx(dtu, rel=1e-12)
    worst = assert_close(g, Ud.cpu().numpy(), U, tol=2e-12, what="vortex 2048^2, one step")
    print(f"vortex {N}^2, one step: worst relative error {worst:.3e}")


def _sums(g, U: np.ndarray) -> np.ndarray:
    avg = g.split(U)["avg"]
    return np.array([avg[k].sum(dtype=np.float64) for k in range(g.ncomp)]) * g.dx * g.dy


def test_vortex_2048_hundred_steps_fp64_and_fp32_stencils(vortex):
    g, U0 = vortex
    s0 = _sums(g, U0)
    out = {}
    for prec in (af.PREC_FP64, af.PREC_MIXED):
        S = af.Solver(g, precision=prec, **KW)
        Ud = S.to_device(U0)
        st, n, t = S.af_run(Ud, 0.0, 1e30, 100, check_every=10)
        assert st == af.AF_OK and n == 100
        assert S.af_check_admissible(Ud) == 0
        U = Ud.cpu().numpy()
        assert np.isfinite(U).all()
        s = _sums(g, U)
        # conservation: each face flux leaves one cell and enters the other;
        # the x- and y-momentum totals are of order one (u = v = 1)
        drift = np.abs(s - s0) / np.maximum(np.abs(s0), 1.0)
        print(f"precision {prec}: t = {t:.6g}, relative drift of the sums {drift.max():.2e}")
        assert drift.max() <= 1e-12
        out[prec] = (U, t)
    (A, ta), (B, tb) = out[af.PREC_FP64], out[af.PREC_MIXED]
    a, b = g.split(A)["avg"], g.split(B)["avg"]
    l1 = np.abs(b - a).sum() / np.abs(a).sum()
    print(f"FP32 stencils against FP64 after 100 steps: relative L1 {l1:.3e}, t {tb:.8g} vs {ta:.8g}")
    assert abs(tb - ta) <= 1e-6 * ta
    assert l1 <= 1e-6
