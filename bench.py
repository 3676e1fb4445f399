#!/usr/bin/env python
"""Benchmark: SSP-RK3 steps of the compact AF method on the 2D viscous shock
tube (1000 x 500 cells, FP64, Re = 200, all limiters) on one MI355X.

A step is one pass of the whole hot path: the CFL time-step reduction and
three limited stages (cell averages and point values).  The timed region is
K steps with the state already resident in HBM, bracketed by device
synchronisation.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-DOF updates/s per RK stage, 2D viscous shock tube; % peak HBM BW; L1 err"
APS = 4  # RK3 attempts per replayed slot of the device-resident step loop
HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6
VALU_SIMDS = 1024      # 256 compute units x 4 SIMDs
# the method's FP64 operations per cell and RK stage in 2D, counted once per
# lattice site from the operators' formulas (primitives, centres, gradients,
# point residual with D^2 and mixed terms, face fluxes, low-order fluxes,
# blends, point low-order update, RK combination): a range, see the design
# notes
ALG_FLOPS_PER_CELL_STAGE = (2600.0, 3300.0)
CLOCK_HZ = 2.4e9
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["paper_2609_29081_amd/csrc/af_stage2d.hip", "paper_2609_29081_amd/csrc/af_device.hpp",
                  "paper_2609_29081_amd/csrc/af_lattice.hpp",
                  "paper_2609_29081_amd/csrc/af_internal.hpp", "paper_2609_29081_amd/build.py"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(g) -> dict:
    """Minimum HBM bytes each kernel kind must move per launch (FP64): its
    inputs read once and its outputs written once, given the stage's data
    layout (see the kernel table in the design notes)."""
    d = 8
    n1, n2 = g.n1, g.n2
    ncell = n1 * n2
    ns = (2 * n1 + 9) * (2 * n2 + 9)              # lattice sites incl. margin
    ngrad = (2 * n1 + 5) * (2 * n2 + 5)
    nring = (n1 + 2) * (n2 + 2)
    nfx, nfy = (n1 + 1) * n2, n1 * (n2 + 1)
    npts = g.state_len // 4 - ncell                # point DOF sites
    face_sites_x = (n1 + 1) * (2 * n2 + 1)         # lattice sites on x-face lines
    face_sites_y = n1 * 0 + (2 * n1 + 1) * (n2 + 1)
    return {
        "lattice": d * (g.state_len + 9 * ns),
        "grad": d * (3 * ns + 6 * ngrad),
        "cellpre": d * (4 * ncell + 18 * nring),
        # one launch per direction; report the mean of the two
        "face": d * 0.5 * (13 * (face_sites_x + face_sites_y) + 2 * 18 * nring + 4 * (nfx + nfy)),
        "cells": d * (4 * (nfx + nfy) + 3 * 4 * ncell),
        "points": d * (15 * ngrad + 2 * 4 * npts),
        "cfl": d * 4 * ncell,
        # fused 2D stage: reads U^(k) and U^n (except the first stage), writes
        # U^(k+1): the mean over the three stages is 8/3 states
        "stage2d": d * g.state_len * 8.0 / 3.0,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n1", type=int, default=1000)
    ap.add_argument("--n2", type=int, default=500)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the all-thread CPU-oracle sample (0 disables the baseline)")
    ap.add_argument("--cpu-seconds-1t", type=float, default=10.0,
                    help="budget of the single-thread CPU-oracle sample (one step at least)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision form")
    ap.add_argument("--no-pexact", action="store_true",
                    help="skip the form with the pressure factor solved exactly")
    ap.add_argument("--roofline-reps", type=int, default=10,
                    help="repetitions of the three stage kinds timed for the roofline")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched shock-tube sweep form")
    ap.add_argument("--batch-n", type=int, default=64,
                    help="instances of the batched shock-tube sweep")
    ap.add_argument("--batch-steps", type=int, default=100,
                    help="accepted steps per instance of the batched sweep")
    ap.add_argument("--no-vortex", action="store_true",
                    help="skip the smooth vortex-wave form (256^2 to 2048^2)")
    ap.add_argument("--vortex-steps", type=int, default=100,
                    help="RK3 steps of each vortex-wave run")
    ap.add_argument("--vortex-sizes", default="256,512,1024,2048",
                    help="vortex-wave grid sizes")
    ap.add_argument("--whole-run", default="",
                    help="also run the 1000 x 500 tube to t = 1 in the listed precisions "
                         "(fp64,mixed; off by default: minutes) and write a summary to "
                         "--whole-run-out")
    ap.add_argument("--whole-run-out", default="",
                    help="markdown file for the whole-run summary")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-blend form")
    ap.add_argument("--learned-train-steps", type=int, default=30000,
                    help="Adam steps of the learned blend's training")
    ap.add_argument("--learned-rows", type=int, default=2000000,
                    help="training rows of the learned blend")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on exactly one GPU; the multi-GPU path (y-slab halo "
              "exchange) is a design only, so --gpus must be 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2609_29081_amd import af
    from paper_2609_29081_amd import workloads as W

    gamma = 1.4
    kw = dict(gamma=gamma, mu=0.005, Pr=0.73, cfl_c=0.2, cfl_v=0.05, limiter=af.LIM_ALL)
    g, f = W.shock_tube_2d(args.n1, args.n2, gamma=gamma)
    U0 = W.make_state(g, f, gamma)
    S = af.Solver(g, **kw)
    dev_U0 = S.to_device(U0)
    U = dev_U0.clone()
    K, Wm = args.steps, args.warmup

    # warm-up (also loads the code objects and builds the step loop's graph)
    if Wm > 0:
        st, ns, _, _ = S.af_run_graph(U, 0.0, 1e30, Wm, attempts_per_slot=APS)
        if st != af.AF_OK:
            raise RuntimeError(f"warm-up failed with status {st}")
        U.copy_(dev_U0)
        st, ns, _ = S.af_run(U, 0.0, 1e30, Wm, check_every=1)

    # timed region: K steps from the initial state, resident in HBM.  Every
    # step decision (the CFL step, accepting an attempt or redoing it with
    # dt/2, as the method prescribes) is taken on the device, and the step
    # rounds are replayed from a HIP graph (af_run_graph)
    U.copy_(dev_U0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    st, nsteps, t_end, attempts = S.af_run_graph(U, 0.0, 1e30, K, attempts_per_slot=APS)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if st != af.AF_OK or nsteps != K:
        raise RuntimeError(f"timed run failed: status {st}, {nsteps}/{K} steps")
    gpu_ms = ev0.elapsed_time(ev1)
    U_graph = U.clone()
    # the same K steps with the decisions on the host (af_run, one
    # synchronisation per attempt), for comparison: the same states
    U.copy_(dev_U0)
    torch.cuda.synchronize()
    eh0 = torch.cuda.Event(enable_timing=True)
    eh1 = torch.cuda.Event(enable_timing=True)
    eh0.record(stream)
    st_h, ns_h, _ = S.af_run(U, 0.0, 1e30, K, check_every=1)
    eh1.record(stream)
    torch.cuda.synchronize()
    host_ms = eh0.elapsed_time(eh1)
    if st_h != af.AF_OK or ns_h != K or not torch.equal(U, U_graph):
        raise RuntimeError("host-decided run differs from the device-decided one")
    sec = gpu_ms / 1e3
    stages = 3 * K
    dof_sites = g.dof_sites
    value = dof_sites * stages / sec
    cell_rate = g.n1 * g.n2 * stages / sec
    stage_ms = gpu_ms / stages
    stage_bytes = 8.0 * g.state_len * 8.0 / 3.0     # mean over the 3 stages: (2+3+3)/3 states
    stage_gbs = stage_bytes / (stage_ms * 1e-3) / 1e9

    # RK3 attempts per accepted step over the same window (a rejected attempt
    # is redone with dt/2; its stages stop at the first flag)
    attempts_per_step = attempts / K
    # the stage launches of the window (host-decided run, timed per launch)
    U.copy_(dev_U0)
    torch.cuda.synchronize()
    S.af_timing(True)
    S.af_timing_read()
    st, _, _ = S.af_run(U, 0.0, 1e30, K, check_every=1)
    kw_ = S.af_timing_read()
    stage_kind = "stage2d" if "stage2d" in kw_ else "lattice"
    # the same kernel over the K steps of the timed window: every launch,
    # the early exits of rejected attempts included (so a shorter mean)
    window = {"launches": kw_[stage_kind][0],
              "avg_launch_us": round(kw_[stage_kind][1] / kw_[stage_kind][0] * 1e3, 3),
              "what": "all stage launches of the timed steps (rejected attempts stop early)"}
    # per-kernel durations of complete stage launches (the three RK3 stage
    # kinds from the initial state at its CFL dt), measured live with HIP
    # events on the launch stream
    from paper_2609_29081_amd.prof_counters import stage_sequence
    S.af_timing_read()
    stage_sequence(S, dev_U0, args.roofline_reps)
    kt = S.af_timing_read()
    S.af_timing(False)
    alg = algorithmic_bytes(g)
    kernels = {}
    for name, (n, ms) in kt.items():
        avg_ms = ms / n
        b = alg.get(name)
        kernels[name] = {"launches": n, "avg_us": round(avg_ms * 1e3, 3),
                         "share": None,
                         "alg_GBs": round(b / (avg_ms * 1e-3) / 1e9, 1) if b else None}
    total = sum(ms for n, ms in kt.values())
    for name, (n, ms) in kt.items():
        kernels[name]["share"] = round(ms / total, 4)
    dom = max(kt.items(), key=lambda kv: kv[1][1])[0]
    dom_avg_s = kt[dom][1] / kt[dom][0] * 1e-3
    achieved = alg[dom] / dom_avg_s / 1e9
    traffic = flops = valu = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("kernel_source_hash") == kernel_source_hash() and tr.get("kernel") == dom \
                and tr.get("n1") == g.n1 and tr.get("n2") == g.n2:
            traffic = tr.get("bytes_per_launch")
            flops = tr.get("fp64_flops_per_launch")
            valu = tr.get("instructions_per_launch", {}).get("SQ_INSTS_VALU")
    # the roof: algorithmic HBM bytes of the dominant kernel per launch (each
    # input read once, each output written once) over its mean launch time.
    # Beside it, the method's algorithmic FP64 flops per cell-stage (the
    # operator-count estimate of the design notes, a range) against the FP64
    # vector peak, and, while the counter file matches the kernel sources, the
    # executed FP64 flops and VALU issue rate from the counters (which include
    # the halo recomputation of the tiles).
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "alg_bytes_per_launch": alg[dom],
                "avg_launch_us": round(dom_avg_s * 1e6, 3), "timed_window": window}
    if dom == "stage2d":
        ncell = g.n1 * g.n2
        lo, hi = (ALG_FLOPS_PER_CELL_STAGE[0] * ncell / dom_avg_s / 1e12,
                  ALG_FLOPS_PER_CELL_STAGE[1] * ncell / dom_avg_s / 1e12)
        roofline["fp64_algorithmic"] = {
            "flops_per_cell_stage": list(ALG_FLOPS_PER_CELL_STAGE),
            "achieved_TFLOPs": [round(lo, 2), round(hi, 2)], "peak": FP64_VALU_PEAK_TFLOPS,
            "frac": [round(lo / FP64_VALU_PEAK_TFLOPS, 4), round(hi / FP64_VALU_PEAK_TFLOPS, 4)]}
    if flops:
        tf = flops / dom_avg_s / 1e12
        ex = {"fp64_flops_per_launch": flops, "TFLOPs": round(tf, 2),
              "frac_of_fp64_peak": round(tf / FP64_VALU_PEAK_TFLOPS, 4),
              "what": "executed FP64 flops (rocprofv3 counters, 64 lanes per wave instruction, "
                      "2 per FMA), halo recomputation included"}
        if valu:
            # a wave64 VALU instruction occupies its SIMD for four cycles
            ex["valu_issue_frac"] = round(valu * 4.0 / (VALU_SIMDS * CLOCK_HZ * dom_avg_s), 4)
            ex["valu_wave_instructions_per_launch"] = valu
        roofline["executed"] = ex

    # CPU baseline: the FP64 oracle on the host cores, first steps of the same
    # workload, and the L1 difference of the GPU after the same steps
    cpu = None
    l1 = None
    if args.cpu_seconds > 0:
        cpu, l1, linf = cpu_baseline(args, g, kw, U0, S, dev_U0, K, dof_sites)
    # the mixed-precision form (FP32 stencils, FP64 blends and updates): the
    # same K steps from t = 0, timed the same way, and its difference from
    # the FP64 form over fixed-dt steps (no halving, equal times)
    forms = {"fp64": {"value": value, "ms_per_step": gpu_ms / K,
                      "stage_us": round(dom_avg_s * 1e6, 1),
                      "step_loop": "af_run_graph: decisions on the device, graph replay"},
             "fp64_host_loop": {"value": dof_sites * stages / (host_ms / 1e3),
                                "ms_per_step": host_ms / K,
                                "step_loop": "af_run: one host synchronisation per attempt",
                                "state": "bitwise equal to the device-decided run"}}
    if not args.no_mixed:
        Sm = af.Solver(g, precision=af.PREC_MIXED, **kw)
        Um = dev_U0.clone()
        if Wm > 0:
            Sm.af_run(Um, 0.0, 1e30, Wm, check_every=1)
        Um.copy_(dev_U0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        if Wm > 0:
            Sm.af_run_graph(Um, 0.0, 1e30, 1, attempts_per_slot=APS)
            Um.copy_(dev_U0)
            torch.cuda.synchronize()
        e0.record(stream)
        stm, nm, _, _ = Sm.af_run_graph(Um, 0.0, 1e30, K, attempts_per_slot=APS)
        e1.record(stream)
        torch.cuda.synchronize()
        if stm != af.AF_OK or nm != K:
            raise RuntimeError(f"mixed run failed: status {stm}, {nm}/{K} steps")
        ms_m = e0.elapsed_time(e1)
        Sm.af_timing(True)
        Sm.af_timing_read()
        stage_sequence(Sm, dev_U0, args.roofline_reps)
        km = Sm.af_timing_read()
        Sm.af_timing(False)
        dt_fix = 0.125 * float(S.af_cfl_dt(dev_U0).item())
        A, B = dev_U0.clone(), dev_U0.clone()
        for n_ in range(10):
            S.af_step(A, dt_fix, n_ * dt_fix)
            Sm.af_step(B, dt_fix, n_ * dt_fix)
        a_, b_ = A.cpu().numpy(), B.cpu().numpy()
        stage_s_m = km["stage2d"][1] / km["stage2d"][0] * 1e-3
        forms["mixed"] = {"value": dof_sites * 3 * K / (ms_m / 1e3), "ms_per_step": ms_m / K,
                          "stage_us": round(stage_s_m * 1e6, 1),
                          "hbm_alg_GBs": round(alg["stage2d"] / stage_s_m / 1e9, 1),
                          "l1_rel_vs_fp64": float(np.abs(b_ - a_).sum() / np.abs(a_).sum()),
                          "linf_rel_vs_fp64": float(np.abs(b_ - a_).max() / np.abs(a_).max()),
                          "l1_rel_vs_fp64_steps": f"10 steps of dt = CFL dt / 8 from t = 0"}
        mfile = os.path.join(ROOT, "profiles", "traffic_mixed.json")
        if os.path.exists(mfile):
            with open(mfile) as fh:
                trm = json.load(fh)
            if trm.get("kernel_source_hash") == kernel_source_hash() and trm.get("n1") == g.n1 \
                    and trm.get("n2") == g.n2:
                f32, f64 = trm["fp32_flops_per_launch"], trm["fp64_flops_per_launch"]
                forms["mixed"].update({
                    "traffic": trm["bytes_per_launch"],
                    "executed_TFLOPs": {"fp32": round(f32 / stage_s_m / 1e12, 2),
                                        "fp64": round(f64 / stage_s_m / 1e12, 2)}})
    if not args.no_pexact:
        forms["pexact"] = pexact_form(g, kw, dev_U0, U_graph, t_end, K, stream)
    if not args.no_vortex:
        forms["vortex_wave"] = vortex_form(args, stream)
    if not args.no_batched:
        forms["batched"] = batched_form(args, stream)
    if not args.no_learned:
        forms["learned"] = learned_form(args, stream)
    out = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": K,
        "warmup": Wm, "ms_per_step": gpu_ms / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"2D viscous shock tube {g.n1}x{g.n2} on [0,1]x[0,0.5], "
                               "rho 120|1.2, p=rho/gamma, mu=0.005 (Re=200), Pr=0.73, "
                               "gamma=1.4, no-slip walls + symmetry top, SSP-RK3, CFL 0.2/0.05, "
                               "all limiters, FP64",
                   "n1": g.n1, "n2": g.n2, "dof_sites": dof_sites, "stages_per_step": 3},
        "cell_updates_per_s": cell_rate,
        "stage_ms": stage_ms,
        "stage_hbm": {"alg_bytes": stage_bytes, "GBs": round(stage_gbs, 1),
                      "frac": round(stage_gbs / HBM_PEAK_GBS, 4)},
        "roofline": roofline,
        "forms": forms,
        "kernels": kernels,
        "rk3_attempts_per_step": round(attempts_per_step, 3),
        "stage_launches_per_s": kw_[stage_kind][0] / sec,
        "cpu_baseline": cpu,
        "l1_err_vs_oracle": l1,
        "linf_rel_vs_oracle": linf if cpu else None,
        "wall_s": wall,
    }
    if args.whole_run:
        out["whole_run"] = whole_run(args, g, U0, kw)
    print(json.dumps(out))
    return 0


def vortex_form(args, stream) -> dict:
    """The smooth density/vortex wave (periodic [0,1]^2, mu = 1e-3,
    Pr = 0.72, all limiters) on n^2 grids, FP64 and mixed precision: K RK3
    steps from t = 0 timed with HIP events (value = DOF sites x 3 x K /
    second), and the stage kernel's mean launch time over complete stage
    launches with its algorithmic HBM bytes (8/3 states per launch) as a
    fraction of the HBM peak.  From 1024^2 on, three states no longer fit in
    the 256 MB last-level cache."""
    import torch

    from paper_2609_29081_amd import af
    from paper_2609_29081_amd import workloads as W
    from paper_2609_29081_amd.prof_counters import stage_sequence

    out = {"workload": f"2D vortex wave (periodic, mu=1e-3, Pr=0.72), {args.vortex_steps} "
                       "RK3 steps from t=0 per run"}
    for n in [int(v) for v in args.vortex_sizes.split(",") if v]:
        print(f"bench: vortex wave {n}^2", file=sys.stderr, flush=True)
        g, f = W.vortex_wave_2d(n)
        U0 = W.make_state(g, f, 1.4)
        rec = {}
        for prec, pname in ((af.PREC_FP64, "fp64"), (af.PREC_MIXED, "mixed")):
            S = af.Solver(g, mu=1e-3, Pr=0.72, cfl_c=0.2, cfl_v=0.05, precision=prec)
            d0 = S.to_device(U0)
            U = d0.clone()
            S.af_run(U, 0.0, 1e30, 2, check_every=1)
            U.copy_(d0)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            st, ns, _ = S.af_run(U, 0.0, 1e30, args.vortex_steps, check_every=1)
            e1.record(stream)
            torch.cuda.synchronize()
            if st != af.AF_OK or ns != args.vortex_steps:
                raise RuntimeError(f"vortex {n} {pname}: status {st}, {ns} steps")
            ms = e0.elapsed_time(e1)
            S.af_timing(True)
            S.af_timing_read()
            stage_sequence(S, d0, 5)
            kt = S.af_timing_read()
            S.af_timing(False)
            st_s = kt["stage2d"][1] / kt["stage2d"][0] * 1e-3
            alg = 8.0 * g.state_len * 8.0 / 3.0
            gbs = alg / st_s / 1e9
            rec[pname] = {"value": g.dof_sites * 3 * args.vortex_steps / (ms / 1e3),
                          "ms_per_step": round(ms / args.vortex_steps, 4),
                          "stage_us": round(st_s * 1e6, 1),
                          "hbm_alg_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
            del S, U, d0
        out[f"{n}x{n}"] = rec
    return out


def pexact_form(g, kw, dev_U0, U_lin, t_lin, K, stream) -> dict:
    """the same K steps from t = 0 with the limiter's pressure factor solved
    from the pressure quadratic (AF_LIM_PEXACT) in place of the linear rule:
    throughput, attempts per step, the time reached, and the final state's
    relative L1 / L-inf difference from the linear rule's run"""
    import numpy as np
    import torch

    from paper_2609_29081_amd import af
    kwe = dict(kw)
    kwe["limiter"] = kw.get("limiter", af.LIM_ALL) | af.LIM_PEXACT
    Se = af.Solver(g, **kwe)
    Ue = dev_U0.clone()
    Se.af_run_graph(Ue, 0.0, 1e30, 1, attempts_per_slot=APS)
    Ue.copy_(dev_U0)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    st, n, t_e, att = Se.af_run_graph(Ue, 0.0, 1e30, K, attempts_per_slot=APS)
    e1.record(stream)
    torch.cuda.synchronize()
    if st != af.AF_OK or n != K:
        raise RuntimeError(f"exact-pressure-rule run failed: status {st}, {n}/{K} steps")
    ms = e0.elapsed_time(e1)
    a, b = U_lin.cpu().numpy(), Ue.cpu().numpy()
    return {"value": g.dof_sites * 3 * K / (ms / 1e3), "ms_per_step": ms / K,
            "rk3_attempts_per_step": round(att / K, 3), "t_reached": t_e,
            "t_reached_linear_rule": t_lin,
            "l1_rel_vs_linear_rule": float(np.abs(b - a).sum() / np.abs(a).sum()),
            "linf_rel_vs_linear_rule": float(np.abs(b - a).max() / np.abs(a).max()),
            "what": "theta^p as the root of the pressure quadratic (AF_LIM_PEXACT), same window"}


def whole_run(args, g, U0, kw) -> dict:
    """The 1000 x 500 tube from t = 0 to t = 1 (the configuration's end
    time), once per listed precision, with the device-resident step loop:
    steps, RK3 attempts per step, GPU time (HIP events around each chunk of
    af_run_graph), DOF
    updates per second over the whole run, the admissibility count at the
    end, and the density along the bottom wall (y = 0) at t = 1."""
    import numpy as np
    import torch

    from paper_2609_29081_amd import af

    res = {}
    lines = []
    for pname in [v for v in args.whole_run.split(",") if v]:
        prec = af.PREC_MIXED if pname == "mixed" else af.PREC_FP64
        S = af.Solver(g, precision=prec, **kw)
        U = S.to_device(U0)
        stream = torch.cuda.current_stream()
        t, steps, attempts, gpu_ms = 0.0, 0, 0, 0.0
        w0 = time.perf_counter()
        last = w0
        status = af.AF_OK
        while t < 1.0:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            status, ns, t, att = S.af_run_graph(U, t, 1.0, 4000, attempts_per_slot=APS)
            e1.record(stream)
            torch.cuda.synchronize()
            gpu_ms += e0.elapsed_time(e1)
            steps += ns
            attempts += att
            if status != af.AF_OK or ns == 0:
                break
            if time.perf_counter() - last > 20:
                last = time.perf_counter()
                print(f"bench: whole run {pname}: step {steps} t {t:.4f} "
                      f"{last - w0:.0f} s", file=sys.stderr, flush=True)
        wall = time.perf_counter() - w0
        bad = S.af_check_admissible(U)
        P = g.split(U.cpu().numpy())
        rho_wall = np.empty(2 * g.n1 + 1)
        rho_wall[0::2] = P["co"][0, 0, :]
        rho_wall[1::2] = P["ye"][0, 0, :]
        r = {"status": int(status), "t_end": t, "steps": steps,
             "rk3_attempts_per_step": round(attempts / max(steps, 1), 3),
             "gpu_s": round(gpu_ms / 1e3, 2), "wall_s": round(wall, 1),
             "value": g.dof_sites * 3 * steps / (gpu_ms / 1e3), "unit": "DOF-updates/s",
             "inadmissible_dofs_at_end": int(bad),
             "wall_density_min_max": [float(rho_wall.min()), float(rho_wall.max())],
             "mass_rel_change": float(P["avg"][0].sum() / g.split(U0)["avg"][0].sum() - 1.0)}
        res[pname] = r
        lines.append(f"| {pname} | {r['status']} | {t:.6f} | {steps} | "
                     f"{r['rk3_attempts_per_step']} | {r['gpu_s']} | {r['wall_s']} | "
                     f"{r['value']:.3e} | {bad} | {r['mass_rel_change']:.2e} |")
        del S, U
    if args.whole_run_out:
        with open(args.whole_run_out, "w") as fh:
            fh.write("# The 2D viscous shock tube 1000x500 (Re = 200) from t = 0 to t = 1\n\n")
            argv = " ".join(a if a != args.whole_run_out else "<file>" for a in sys.argv[1:])
            fh.write(f"Command: `python bench.py {argv}`\n\n")
            fh.write("| precision | status | t reached | steps | RK3 attempts per step | GPU s "
                     "| wall s | DOF-updates/s | inadmissible DOFs at end | mass change |\n")
            fh.write("|---|---|---|---|---|---|---|---|---|---|\n")
            fh.write("\n".join(lines) + "\n")
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, g, kw, U0, S, dev_U0, K, dof_sites):
    """The FP64 oracle on the host: on all its threads over the first steps
    of the timed window (all K of them when they fit in --cpu-seconds), and
    on one thread over as many of those steps as fit in --cpu-seconds-1t
    (at least one).  Returns the record, and the L1 / relative L-inf
    difference of the GPU state after the same all-thread steps."""
    import numpy as np

    import oracle as O
    cfg = O.make_cfg(g, **{k: v for k, v in kw.items()})
    nthreads = O.threads()

    def sample(budget, max_steps):
        Uc = U0.copy()
        n, spent, t_sim = 0, 0.0, 0.0
        while n < max_steps and (n == 0 or spent < budget):
            c0 = time.perf_counter()
            _, dtu, _, _ = O.step(cfg, Uc, 0.0, t_sim)
            spent += time.perf_counter() - c0
            t_sim += dtu
            n += 1
        return Uc, n, spent

    print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
    Uc, n_all, t_all = sample(args.cpu_seconds, K)
    O.set_threads(1)
    try:
        _, n_one, t_one = sample(args.cpu_seconds_1t, K)
    finally:
        O.set_threads(nthreads)
    # the GPU over the same steps, for the comparison and its rate there
    import torch
    Ug = dev_U0.clone()
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    st, ns2, _ = S.af_run(Ug, 0.0, 1e30, n_all, check_every=1)
    torch.cuda.synchronize()
    g_s = time.perf_counter() - g0
    Pg, Pc = g.split(Ug.cpu().numpy()), g.split(Uc)
    l1 = float(np.abs(Pg["avg"][0] - Pc["avg"][0]).sum() * g.dx * g.dy)
    linf = max(float(np.abs(Pg[n][k] - Pc[n][k]).max() / np.abs(Pc[n][k]).max())
               for n in Pg for k in range(4))
    cpu = {"value": dof_sites * 3 * n_all / t_all, "unit": "DOF-updates/s",
           "cores": nthreads, "kind": "oracle",
           "sample": f"steps 1-{n_all} of the timed window ({g.n1}x{g.n2} shock tube from t=0, "
                     f"whole grid) on {nthreads} threads, {t_all:.1f} s",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "single_thread": {"value": dof_sites * 3 * n_one / t_one, "unit": "DOF-updates/s",
                             "sample": f"steps 1-{n_one} on one thread, {t_one:.1f} s"},
           "gpu_same_steps_wall": {"value": dof_sites * 3 * n_all / g_s,
                                   "what": f"the GPU over the same {n_all} steps, host wall "
                                           "clock around af_run"}}
    return cpu, l1, linf


def learned_form(args, stream) -> dict:
    """The learned-blend form.

    Training data: features and theta^s of every face of the 1000 x 500
    shock tube (FP64, plain limiter) after steps 1, 2, 3, 5, 10, 20, 50,
    100, 200 and 400 (10.0 M faces; the first steps, where the diaphragm's
    jump turns into a viscous shock, are where the blend acts most); a tenth
    held out; from the rest a training set of --learned-rows rows (every
    face with theta^s < 0.999 and random others, workloads.balanced_rows).
    Training: Adam (minibatches of 1024) from the seeded initial weights,
    the learning rate stepped down over the run: 2e-3 for the first two
    thirds of the steps, 5e-4 for the next sixth, 1.25e-4 for the last.

    Evaluation, each run timed with HIP events (value = DOF sites x 3 x
    accepted steps / second):
    * equal error: the 500 x 250 tube from t = 0 to t = 1e-3 with the plain
      limiter, the learned blend, the untrained network and no smoothness
      blend, each with its L1 density error against the plain 1000 x 500 run
      averaged onto the 500 x 250 cells (2 x 2 cell averages are exact);
    * the 2048 x 1024 tube from t = 0 to t = 1e-4 and the 1000 x 500 tube to
      the same time, with the L1 density distance of each form from the
      plain run of its grid."""
    import numpy as np
    import torch

    from paper_2609_29081_amd import af
    from paper_2609_29081_amd import workloads as W

    gamma = 1.4
    kw = dict(gamma=gamma, mu=0.005, Pr=0.73, cfl_c=0.2, cfl_v=0.05)
    dev = torch.device("cuda:0")
    print("bench: learned blend, training data", file=sys.stderr, flush=True)
    g3, f3 = W.shock_tube_2d(1000, 500, gamma=gamma)
    S3 = af.Solver(g3, limiter=af.LIM_ALL, **kw)
    U = S3.to_device(W.make_state(g3, f3, gamma))
    Xs, ys, done = [], [], 0
    tmp = torch.empty_like(U)
    snaps = (1, 2, 3, 5, 10, 20, 50, 100, 200, 400)
    for target in snaps:
        st, n, _, _ = S3.af_run_graph(U, 0.0, 1e30, target - done)
        if st != af.AF_OK:
            raise RuntimeError(f"training-data run failed: {st}")
        done = target
        Xs.append(S3.af_blend_features(U))
        ts = torch.empty(S3.face_count, dtype=torch.float32, device=dev)
        S3.af_rk_stage_blend(0, None, U, tmp, dt=0.0, theta_s_out=ts)
        ys.append(ts)
    del S3, U, tmp
    X, y = torch.cat(Xs), torch.cat(ys)
    del Xs, ys
    # a held-out tenth of the faces; the training rows come from the rest
    perm = torch.randperm(X.shape[0], generator=torch.Generator().manual_seed(0)).to(dev)
    X, y = X[perm].contiguous(), y[perm].contiguous()
    nhold = X.shape[0] // 10
    Xh, yh = X[:nhold].contiguous(), y[:nhold].contiguous()
    idx = torch.as_tensor(W.balanced_rows(y[nhold:].cpu().numpy(), seed=0,
                                          total=args.learned_rows), device=dev) + nhold
    Xt, yt = X[idx].contiguous(), y[idx].contiguous()
    del X, y
    P0 = torch.as_tensor(W.mlp_init(0), device=dev)
    P = P0.clone()
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    _, l0 = af.mlp_grad(Xh, yh, P)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nsteps = args.learned_train_steps
    done = 0
    for frac, lr in ((2 / 3, 2e-3), (5 / 6, 5e-4), (1.0, 1.25e-4)):
        upto = int(round(frac * nsteps))
        if upto > done:
            af.mlp_train(Xt, yt, P, m, v, done, upto - done, 1024, lr)
            done = upto
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    _, l1 = af.mlp_grad(Xh, yh, P)
    frac_lt1 = float((yh < 0.999).float().mean().item())
    low = torch.nonzero(yh < 0.999).flatten()
    _, l_low = af.mlp_grad(Xh[low].contiguous(), yh[low].contiguous(), P)
    rmse_low = float(l_low.item()) ** 0.5
    rmse_one = float(((1.0 - yh[low]) ** 2).mean().item()) ** 0.5
    ntrain = int(Xt.shape[0])
    del Xt, yt, Xh, yh

    forms = (("plain", af.LIM_ALL, None),
             ("learned", af.LIM_ALL | af.LIM_LEARNED, P),
             ("untrained", af.LIM_ALL | af.LIM_LEARNED, P0),
             ("no_smoothness", af.LIM_PP | af.LIM_POINT | af.LIM_CENTRE, None))

    def evaluate(gg, UU, t_final, names=None):
        runs = {}
        for name, lim, net in forms:
            if names and name not in names:
                continue
            S = af.Solver(gg, limiter=lim, **kw)
            if net is not None:
                S.af_set_blend_net(net)
            Ud = S.to_device(UU)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            # the learned blend needs the host-decided loop (its inference
            # runs before each stage)
            st, n, t = S.af_run(Ud, 0.0, t_final, 10 ** 6, check_every=1)
            e1.record(stream)
            torch.cuda.synchronize()
            if st != af.AF_OK:
                raise RuntimeError(f"{name} run failed: {st}")
            ms = e0.elapsed_time(e1)
            runs[name] = (gg.split(Ud.cpu().numpy())["avg"][0], n, ms)
            del S, Ud
        return runs

    out = {"workload": "2D viscous shock tube (Re=200, FP64), plain limiter against the learned "
                       "blend; network trained on theta^s of the 1000x500 tube after steps "
                       + ", ".join(str(k) for k in snaps),
           "train": {"samples": ntrain, "held_out": nhold, "steps": args.learned_train_steps,
                     "batch": 1024, "lr": [2e-3, 5e-4, 1.25e-4],
                     "lr_until_step": [int(round(f * nsteps)) for f in (2 / 3, 5 / 6, 1.0)],
                     "seconds": round(train_s, 2),
                     "loss_held_out_before": float(l0.item()),
                     "loss_held_out_after": float(l1.item()),
                     "fraction_theta_s_below_1": round(frac_lt1, 4),
                     "rmse_held_out_where_theta_s_below_1": round(rmse_low, 5),
                     "rmse_of_constant_1_there": round(rmse_one, 5)}}
    # equal error: 500 x 250 against the plain 1000 x 500 run averaged onto it
    print("bench: learned blend, equal-error runs", file=sys.stderr, flush=True)
    te = 1e-3
    ref_runs = evaluate(g3, W.make_state(g3, f3, gamma), te, names=("plain",))
    rho_f = ref_runs["plain"][0]
    rho_ref = 0.25 * (rho_f[0::2, 0::2] + rho_f[1::2, 0::2] + rho_f[0::2, 1::2] + rho_f[1::2, 1::2])
    gc, fc = W.shock_tube_2d(500, 250, gamma=gamma)
    runs_c = evaluate(gc, W.make_state(gc, fc, gamma), te)
    eq = {"grid": "500x250", "t": te, "reference": "plain 1000x500 run, 2x2 cell averages"}
    for name, (rho, n, ms) in runs_c.items():
        eq[name] = {"value": gc.dof_sites * 3 * n / (ms / 1e3), "steps": n, "ms": round(ms, 1),
                    "l1_rho_err": float(np.abs(rho - rho_ref).sum() * gc.dx * gc.dy)}
    out["equal_error"] = eq
    print("bench: learned blend, 2048x1024 runs", file=sys.stderr, flush=True)
    t_final = 1e-4
    g5, f5 = W.shock_tube_2d(2048, 1024, gamma=gamma)
    runs = evaluate(g5, W.make_state(g5, f5, gamma), t_final)
    rho_plain = runs["plain"][0]
    for name, (rho, n, ms) in runs.items():
        out[name] = {"value": g5.dof_sites * 3 * n / (ms / 1e3), "unit": "DOF-updates/s",
                     "steps": n, "ms": round(ms, 1),
                     "l1_rho_vs_plain": float(np.abs(rho - rho_plain).sum() * g5.dx * g5.dy)}
    # the same comparison at the training grid (1000 x 500, to the same t)
    runs3 = evaluate(g3, W.make_state(g3, f3, gamma), t_final)
    out["at_1000x500"] = {name: {"steps": n, "l1_rho_vs_plain": float(
        np.abs(rho - runs3["plain"][0]).sum() * g3.dx * g3.dy)} for name, (rho, n, ms) in runs3.items()}
    out["value"] = out["learned"]["value"]
    return out


def batched_form(args, stream) -> dict:
    """The batched form: a seeded sweep of viscous shock tubes (random
    Reynolds number, density ratio and grid, see workloads.shock_tube_sweep),
    mixed precision, advanced together by af_batch_run with HIP-graph replay,
    each instance with its own time step and halving; the stage variant (tile
    shape) is chosen by af_batch_tune on the initial states.  Timed: K
    accepted steps of every instance from t = 0 (inputs resident in HBM).
    value = sum over instances of DOF sites x 3 stages x steps / second."""
    import torch

    from paper_2609_29081_amd import af
    from paper_2609_29081_amd import workloads as W

    print(f"bench: batched sweep of {args.batch_n} shock tubes", file=sys.stderr, flush=True)
    insts = W.shock_tube_sweep(args.batch_n, seed=0)
    solvers = [af.Solver(g, precision=af.PREC_MIXED, cfl_c=0.2, cfl_v=0.05,
                         limiter=af.LIM_ALL, **kw) for g, f, kw in insts]
    init = [S.to_device(W.make_state(g, f, kw["gamma"])) for S, (g, f, kw) in zip(solvers, insts)]
    states = [U.clone() for U in init]
    B = af.Batch(solvers)
    t0 = time.perf_counter()
    us = B.af_batch_tune(states, 0.0, 1e30, reps=3)
    tune_s = time.perf_counter() - t0
    names = af.stage_variants()
    chosen = names[B.variant]
    K, Wm = args.batch_steps, min(args.warmup, 2)
    if Wm > 0:
        B.af_batch_run(states, 0.0, 1e30, Wm, attempts_per_slot=4, use_graph=True)
        for U, U0 in zip(states, init):
            U.copy_(U0)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    st, n, t, att = B.af_batch_run(states, 0.0, 1e30, K, attempts_per_slot=4, use_graph=True,
                                   stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    if st != [af.AF_OK] * len(insts) or n != [K] * len(insts):
        raise RuntimeError(f"batched run failed: status {st}, steps {n}")
    ms = e0.elapsed_time(e1)
    dof = sum(g.dof_sites for g, f, kw in insts)
    cells = sum(g.n1 * g.n2 for g, f, kw in insts)
    return {"value": dof * 3 * K / (ms / 1e3), "unit": "DOF-updates/s",
            "cell_updates_per_s": cells * 3 * K / (ms / 1e3),
            "ms_total": round(ms, 1), "wall_s": round(wall, 2),
            "workload": f"{len(insts)} viscous shock tubes, rng seed 0: Re ~ U[200,1000], "
                        "density ratio ~ U[50,200], N1 on {128,...,1024} step 64, N2 = N1/2; "
                        f"{K} accepted steps each, own dt and halving; mixed precision",
            "instances": len(insts), "cells": cells, "dof_sites": dof,
            "rk3_attempts_per_step": round(sum(att) / (K * len(insts)), 3),
            "graph": True, "attempts_per_slot": 4,
            "variant": chosen[0], "tile": f"16x{chosen[2]}",
            "tune_us_per_slot": {nm[0]: round(u, 1) for nm, u in zip(names, us) if u > 0},
            "tune_s": round(tune_s, 2),
            "error": "bitwise equal to single-instance mixed runs; FP32-stencil error as in "
                     "the mixed form"}


if __name__ == "__main__":
    sys.exit(main())
