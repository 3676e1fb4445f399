"""Writes shock_tube_200x100_t1.txt: the FP64 oracle's solution of the 2D
viscous shock tube of Sec. 4 (Daru-Tenaud setting at Re = 200: rho 120 | 1.2,
p = rho/gamma, at rest, no-slip adiabatic walls at x = 0, 1 and y = 0,
symmetry at y = 0.5, Pr = 0.73, gamma = 1.4, all limiters, SSP-RK3 with
C^c = 0.2, C^v = 0.05) on 200 x 100 cells at t = 1.

Calls only oracle/ (and the input generator).  Stored: the step count and
halvings, the density of the point values along the bottom wall y = 0
(corners and y-edge midpoints, x = 0, dx/2, ..., 1), and the integrals of
the four conserved variables over the cell averages.

    python tests/golden/make_shock_tube_t1.py [--npy PATH]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2609_29081_amd import workloads as W  # noqa: E402

N1, N2, T_END = 200, 100, 1.0
OUT = os.path.join(HERE, "shock_tube_200x100_t1.txt")


def wall_density(g, U):
    P = g.split(U)
    rho = np.empty(2 * g.n1 + 1)
    rho[0::2] = P["co"][0, 0, :]
    rho[1::2] = P["ye"][0, 0, :]
    return rho


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--npy", default=None, help="also save the whole final state here")
    a = ap.parse_args()
    g, f = W.shock_tube_2d(N1, N2)
    U = W.make_state(g, f, 1.4)
    c = O.make_cfg(g, mu=0.005, Pr=0.73, cfl_c=0.2, cfl_v=0.05)
    t, steps, halv = 0.0, 0, 0
    t0 = time.time()
    while t < T_END:
        st, dtu, h, fl = O.step(c, U, 0.0, t, T_END)
        if st != 0:
            raise RuntimeError(f"oracle step failed at t={t}")
        t += dtu
        steps += 1
        halv += h
        if steps % 500 == 0:
            print(f"step {steps} t {t:.5f} halvings {halv} {time.time() - t0:.0f} s", flush=True)
    avg = g.split(U)["avg"]
    integ = avg.sum(axis=(1, 2)) * g.dx * g.dy
    rho = wall_density(g, U)
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle, 2D viscous shock tube (Sec. 4) at Re=200, 200x100 cells, t=1\n")
        fh.write("# SSP-RK3, CFL 0.2 / 0.05, all limiters; written by make_shock_tube_t1.py\n")
        fh.write(f"steps {steps}\nhalvings {halv}\nt {t!r}\n")
        fh.write("integrals " + " ".join(repr(float(v)) for v in integ) + "\n")
        fh.write("# wall density at x = k dx/2, k = 0..400\n")
        for v in rho:
            fh.write(f"{float(v)!r}\n")
    if a.npy:
        np.save(a.npy, U)
    print(f"done: {steps} steps, {halv} halvings, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
