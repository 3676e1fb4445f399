"""af_run_graph (every step decision on the device, graph replay) against
af_run (host decisions): the same method, so the same steps, halvings,
final time and state, bit for bit, in both precisions; and the same failure
when the halving budget runs out (the remark on the time step at the end of
Sec. 3.4)."""
import pytest

from paper_2609_29081_amd import workloads as W

pytestmark = pytest.mark.gpu


def solver(g, **kw):
    from paper_2609_29081_amd import af
    return af.Solver(g, mu=0.005, Pr=0.73, cfl_c=0.2, cfl_v=0.05, device="cuda:0", **kw)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("t_final,steps", [(1e30, 25), (4e-3, 1000)])
def test_run_graph_equals_run(precision, t_final, steps):
    import torch

    from paper_2609_29081_amd import af
    g, f = W.shock_tube_2d(64, 32)
    U0 = W.make_state(g, f, 1.4)
    S = solver(g, precision=precision)
    A, B = S.to_device(U0), S.to_device(U0)
    print(f"run_graph: precision {precision}, t_final {t_final}, {steps} steps", flush=True)
    sa, na, ta = S.af_run(A, 0.0, t_final, steps, check_every=1)
    sb, nb, tb, att = S.af_run_graph(B, 0.0, t_final, steps, attempts_per_slot=3)
    torch.cuda.synchronize()
    assert sa == sb == af.AF_OK
    assert na == nb and ta == tb and att >= nb
    assert torch.equal(A, B)


def test_run_graph_reports_exhausted_halving_like_run():
    import torch

    from paper_2609_29081_amd import af
    g, f = W.shock_tube_2d(48, 24)
    U0 = W.make_state(g, f, 1.4)
    # no halving allowed: the first rejected attempt ends both runs
    S = solver(g, max_halvings=0)
    A, B = S.to_device(U0), S.to_device(U0)
    sa, na, ta = S.af_run(A, 0.0, 1e30, 200, check_every=1)
    sb, nb, tb, att = S.af_run_graph(B, 0.0, 1e30, 200)
    torch.cuda.synchronize()
    assert sa == sb == af.AF_E_PP
    assert na == nb and ta == tb
    assert torch.equal(A, B)
