"""af_step_noalloc: af_step on the library's own scratch array.

It must give exactly what af_step gives with a caller workspace (the same
kernels on the same data), also when a call follows one on a larger grid
whose contents the array still holds, and it must refuse grids whose
workspace exceeds the array before any device work.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2609_29081_amd import af
from paper_2609_29081_amd import workloads as W

SCRATCH = 16 << 20  # AF_NOALLOC_SCRATCH_BYTES


def test_noalloc_rejects_grids_beyond_the_scratch_array():
    g, _ = W.shock_tube_2d(1000, 500)
    p = af.Params()
    assert af.lib().af_default_params(C.byref(p)) == af.AF_OK
    p.n1, p.n2, p.x1, p.y1 = g.n1, g.n2, g.x1, g.y1
    h = C.c_void_p()
    assert af.lib().af_init_grid(C.byref(p), C.byref(h)) == af.AF_OK
    try:
        assert af.lib().af_workspace_bytes(h) > SCRATCH
        dtu, hv = C.c_double(), C.c_int()
        st = af.lib().af_step_noalloc(h, C.c_void_p(8), None, 0.0, 0.0, 1.0, C.byref(dtu),
                                      C.byref(hv))
        assert st == af.AF_E_ARG
        assert b"scratch" in af.lib().af_last_error()
        st = af.lib().af_step_noalloc(h, None, None, 0.0, 0.0, 1.0, None, None)
        assert st == af.AF_E_ARG
    finally:
        af.lib().af_destroy(h)


def cases():
    # the second call is on a smaller grid than the first; then 1D
    g, f = W.shock_tube_2d(64, 32)
    yield g, f, dict(mu=0.005, Pr=0.73)
    g, f = W.shock_tube_2d(40, 20)
    yield g, f, dict(mu=0.005, Pr=0.73)
    g, f = W.leblanc_1d(96)
    yield g, f, dict(mu=1e-3, Pr=0.75)


@pytest.mark.gpu
def test_noalloc_step_equals_af_step():
    import torch
    for g, f, phys in cases():
        U = W.make_state(g, f, 1.4)
        S = af.Solver(g, device="cuda:0", **phys)
        assert S.ws_bytes <= SCRATCH
        A, B = S.to_device(U), S.to_device(U)
        t = 0.0
        print(f"noalloc: grid {g.n1}x{g.n2} dim {g.dim}", flush=True)
        for _ in range(3):
            sa, dta, ha = S.af_step(A, t=t)
            sb, dtb, hb = S.af_step_noalloc(B, t=t)
            torch.cuda.synchronize()
            assert sa == sb == af.AF_OK
            assert dta == dtb and ha == hb
            assert torch.equal(A, B), float((A - B).abs().max())
            t += dta
        assert np.isfinite(B.cpu().numpy()).all()
