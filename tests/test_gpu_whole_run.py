"""The 2D viscous shock tube (Sec. 4 setting at Re = 200) run to its end
time t = 1 on the GPU, against the FP64 oracle's run of the same problem
(tests/golden/shock_tube_200x100_t1.txt, written by make_shock_tube_t1.py
from oracle/ alone).

Both runs take thousands of steps with their own CFL time steps and halving
decisions, so differences of rounding order (the stage parity bar is 1e-12
per stage) are carried and amplified by the flow over the whole run; the
comparison is therefore of what the run must get right: the same number of
steps and halvings, positivity of every DOF at t = 1 (the theorem at the end
of Sec. 3.4), mass conserved to round-off (no mass flux through walls and the
symmetry line), and the density along the bottom wall and the integrals of
the conserved variables within a relative 1e-6 of the oracle's.
"""
import os

import numpy as np
import pytest

from paper_2609_29081_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "shock_tube_200x100_t1.txt")


def read_golden():
    meta, rho = {}, []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            parts = line.split()
            if len(parts) == 1:
                rho.append(float(parts[0]))
            else:
                meta[parts[0]] = [float(v) for v in parts[1:]]
    return meta, np.array(rho)


def test_golden_file_is_consistent():
    meta, rho = read_golden()
    assert rho.shape == (401,) and rho.min() > 0
    assert meta["t"][0] == 1.0
    # mass of the initial state: 120 x 0.25 + 1.2 x 0.25
    assert abs(meta["integrals"][0] - 30.3) < 1e-10


@pytest.mark.gpu
def test_shock_tube_to_t1_matches_oracle_run():
    import torch

    from paper_2609_29081_amd import af
    meta, rho_ref = read_golden()
    g, f = W.shock_tube_2d(200, 100)
    S = af.Solver(g, mu=0.005, Pr=0.73, cfl_c=0.2, cfl_v=0.05, device="cuda:0")
    U = S.to_device(W.make_state(g, f, 1.4))
    print("whole run: 200x100 shock tube to t=1", flush=True)
    st, ns, t = S.af_run(U, 0.0, 1.0, 10 ** 6, check_every=1)
    torch.cuda.synchronize()
    assert st == af.AF_OK and t == 1.0
    assert S.af_check_admissible(U) == 0
    P = g.split(U.cpu().numpy())
    integ = P["avg"].sum(axis=(1, 2)) * g.dx * g.dy
    rho = np.empty(401)
    rho[0::2] = P["co"][0, 0, :]
    rho[1::2] = P["ye"][0, 0, :]
    d_rho = float(np.abs(rho - rho_ref).max() / np.abs(rho_ref).max())
    d_int = [float(abs(a - b) / max(abs(b), 1e-300)) for a, b in zip(integ, meta["integrals"])]
    print(f"steps {ns} (oracle {int(meta['steps'][0])}), wall density rel diff {d_rho:.3e}, "
          f"integrals rel diff {d_int}", flush=True)
    assert ns == int(meta["steps"][0])
    assert abs(integ[0] - 30.3) < 1e-11
    assert d_rho < 1e-6
    assert max(d_int) < 1e-6
