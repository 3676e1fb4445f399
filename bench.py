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
HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6
VALU_SIMDS = 1024      # 256 compute units x 4 SIMDs
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
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the CPU-oracle baseline sample (0 disables it)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision form")
    ap.add_argument("--roofline-reps", type=int, default=10,
                    help="repetitions of the three stage kinds timed for the roofline")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched shock-tube sweep form")
    ap.add_argument("--batch-n", type=int, default=64,
                    help="instances of the batched shock-tube sweep")
    ap.add_argument("--batch-steps", type=int, default=100,
                    help="accepted steps per instance of the batched sweep")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-blend form")
    ap.add_argument("--learned-train-steps", type=int, default=20000,
                    help="Adam steps of the learned blend's training")
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

    # warm-up (also loads the code objects)
    if Wm > 0:
        st, ns, _ = S.af_run(U, 0.0, 1e30, Wm, check_every=1)
        if st != af.AF_OK:
            raise RuntimeError(f"warm-up failed with status {st}")

    # timed region: K steps from the initial state, resident in HBM
    U.copy_(dev_U0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    # the flags are checked after every step (a rejected step is redone with
    # dt/2 at once, as the method prescribes); one host synchronisation per step
    st, nsteps, t_end = S.af_run(U, 0.0, 1e30, K, check_every=1)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if st != af.AF_OK or nsteps != K:
        raise RuntimeError(f"timed run failed: status {st}, {nsteps}/{K} steps")
    gpu_ms = ev0.elapsed_time(ev1)
    sec = gpu_ms / 1e3
    stages = 3 * K
    dof_sites = g.dof_sites
    value = dof_sites * stages / sec
    cell_rate = g.n1 * g.n2 * stages / sec
    stage_ms = gpu_ms / stages
    stage_bytes = 8.0 * g.state_len * 8.0 / 3.0     # mean over the 3 stages: (2+3+3)/3 states
    stage_gbs = stage_bytes / (stage_ms * 1e-3) / 1e9

    # RK3 attempts per accepted step over the same window (a rejected attempt
    # is redone with dt/2; its stages stop at the first flag): launch counts
    U.copy_(dev_U0)
    torch.cuda.synchronize()
    S.af_timing(True)
    S.af_timing_read()
    st, _, _ = S.af_run(U, 0.0, 1e30, K, check_every=1)
    kw_ = S.af_timing_read()
    stage_kind = "stage2d" if "stage2d" in kw_ else "lattice"
    attempts_per_step = kw_[stage_kind][0] / (3.0 * K)
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
    hbm = {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": alg[dom]}
    if flops:
        # the stage executes ~20 FP64 flops per algorithmic byte, twice the
        # FP64 ridge: the FP64 VALU is the binding roof
        tf = flops / dom_avg_s / 1e12
        roofline = {"bound": "alu", "kernel": dom, "achieved": round(tf, 2),
                    "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(tf / FP64_VALU_PEAK_TFLOPS, 4), "traffic": traffic,
                    "flops_per_launch": flops,
                    "flops_kind": "executed FP64 flops (rocprofv3 counters, 64 lanes per wave "
                                  "instruction), an upper bound on the algorithmic count",
                    "avg_launch_us": round(dom_avg_s * 1e6, 3), "hbm": hbm,
                    "timed_window": window}
        if valu:
            # issue rate of all VALU wave instructions (a wave64 instruction
            # occupies its SIMD for four cycles; 1024 SIMDs at 2.4 GHz)
            roofline["valu_issue"] = {
                "wave_instructions_per_launch": valu,
                "frac": round(valu * 4.0 / (VALU_SIMDS * CLOCK_HZ * dom_avg_s), 4),
                "what": "all VALU wave instructions (counters) x 4 cycles / (SIMDs x clock x "
                        "launch time)"}
    else:
        roofline = dict({"bound": "hbm", "kernel": dom, "traffic": traffic,
                         "avg_launch_us": round(dom_avg_s * 1e6, 3), "timed_window": window},
                        **hbm)

    # CPU baseline: the FP64 oracle on the host cores, first steps of the same
    # workload, and the L1 difference of the GPU after the same steps
    cpu = None
    l1 = None
    if args.cpu_seconds > 0:
        import oracle as O
        cfg = O.make_cfg(g, **{k: v for k, v in kw.items()})
        Uc = U0.copy()
        n_cpu, t_cpu, t_sim = 0, 0.0, 0.0
        while t_cpu < args.cpu_seconds and n_cpu < 50:
            c0 = time.perf_counter()
            stc, dtu, h, fl = O.step(cfg, Uc, 0.0, t_sim)
            t_cpu += time.perf_counter() - c0
            t_sim += dtu
            n_cpu += 1
        cpu = {"value": dof_sites * 3 * n_cpu / t_cpu, "unit": "DOF-updates/s",
               "cores": O.threads(), "kind": "oracle",
               "sample": f"first {n_cpu} RK3 steps of the {g.n1}x{g.n2} shock tube from t=0 "
                         f"(whole grid, {t_cpu:.1f} s)"}
        Ug = dev_U0.clone()
        st, ns2, _ = S.af_run(Ug, 0.0, 1e30, n_cpu, check_every=1)
        Pg, Pc = g.split(Ug.cpu().numpy()), g.split(Uc)
        l1 = float(np.abs(Pg["avg"][0] - Pc["avg"][0]).sum() * g.dx * g.dy)
        linf = max(float(np.abs(Pg[n][k] - Pc[n][k]).max() / np.abs(Pc[n][k]).max())
                   for n in Pg for k in range(4))
    # the mixed-precision form (FP32 stencils, FP64 blends and updates): the
    # same K steps from t = 0, timed the same way, and its difference from
    # the FP64 form over fixed-dt steps (no halving, equal times)
    forms = {"fp64": {"value": value, "ms_per_step": gpu_ms / K,
                      "stage_us": round(dom_avg_s * 1e6, 1)}}
    if not args.no_mixed:
        Sm = af.Solver(g, precision=af.PREC_MIXED, **kw)
        Um = dev_U0.clone()
        if Wm > 0:
            Sm.af_run(Um, 0.0, 1e30, Wm, check_every=1)
        Um.copy_(dev_U0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        stm, nm, _ = Sm.af_run(Um, 0.0, 1e30, K, check_every=1)
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
    print(json.dumps(out))
    return 0


def learned_form(args, stream) -> dict:
    """The learned-blend form.  Training data: features and theta^s of every
    face of the 1000 x 500 shock tube (FP64, plain limiter) after steps 1,
    2, 3, 5, 10, 20 and 50 (7.0 M faces; the first steps, where the
    diaphragm's jump turns into a viscous shock, are where the blend acts
    most; a tenth held out, the rest balanced by workloads.balanced_rows); training: Adam (lr 2e-3, minibatches of 1024)
    from the seeded initial weights.  Evaluation on the 2048 x 1024 shock tube
    (FP64, Re = 200) from t = 0 to t = 1e-4: the plain limiter, the learned
    blend (AF_LIM_LEARNED: the network's theta_nn in place of theta^s, then
    the density/pressure limiter), the untrained network, and no smoothness
    blend at all (theta^s = 1).  Each run is
    timed with HIP events; value = DOF sites x 3 x accepted steps / second.
    The plain limiter judges the error: L1 = sum |rho - rho_plain| dx dy of
    the cell averages at t = 1e-4."""
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
    for target in (1, 2, 3, 5, 10, 20, 50):
        st, n, _ = S3.af_run(U, 0.0, 1e30, target - done, check_every=1)
        if st != af.AF_OK:
            raise RuntimeError(f"training-data run failed: {st}")
        done = target
        Xs.append(S3.af_blend_features(U))
        ts = torch.empty(S3.face_count, dtype=torch.float32, device=dev)
        S3.af_rk_stage_blend(0, None, U, tmp, dt=0.0, theta_s_out=ts)
        ys.append(ts)
    X, y = torch.cat(Xs), torch.cat(ys)
    # a held-out tenth of the faces; the training rows are every face of the
    # rest where theta^s < 0.999 and three times as many of the others
    perm = torch.randperm(X.shape[0], generator=torch.Generator().manual_seed(0)).to(dev)
    X, y = X[perm].contiguous(), y[perm].contiguous()
    nhold = X.shape[0] // 10
    Xh, yh = X[:nhold], y[:nhold]
    idx = torch.as_tensor(W.balanced_rows(y[nhold:].cpu().numpy(), seed=0), device=dev) + nhold
    Xt, yt = X[idx].contiguous(), y[idx].contiguous()
    P0 = torch.as_tensor(W.mlp_init(0), device=dev)
    P = P0.clone()
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    _, l0 = af.mlp_grad(Xh, yh, P)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    af.mlp_train(Xt, yt, P, m, v, 0, args.learned_train_steps, 1024, 2e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    _, l1 = af.mlp_grad(Xh, yh, P)
    frac_lt1 = float((yh < 0.999).float().mean().item())
    low = torch.nonzero(yh < 0.999).flatten()
    _, l_low = af.mlp_grad(Xh[low].contiguous(), yh[low].contiguous(), P)
    rmse_low = float(l_low.item()) ** 0.5
    rmse_one = float(((1.0 - yh[low]) ** 2).mean().item()) ** 0.5

    t_final = 1e-4

    def evaluate(gg, UU):
        runs = {}
        for name, lim, net in (("plain", af.LIM_ALL, None),
                               ("learned", af.LIM_ALL | af.LIM_LEARNED, P),
                               ("untrained", af.LIM_ALL | af.LIM_LEARNED, P0),
                               ("no_smoothness", af.LIM_PP | af.LIM_POINT | af.LIM_CENTRE, None)):
            S = af.Solver(gg, limiter=lim, **kw)
            if net is not None:
                S.af_set_blend_net(net)
            Ud = S.to_device(UU)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            st, n, t = S.af_run(Ud, 0.0, t_final, 10 ** 6, check_every=1)
            e1.record(stream)
            torch.cuda.synchronize()
            if st != af.AF_OK:
                raise RuntimeError(f"{name} run failed: {st}")
            ms = e0.elapsed_time(e1)
            runs[name] = (gg.split(Ud.cpu().numpy())["avg"][0], n, ms)
            del S, Ud
        return runs

    print("bench: learned blend, 2048x1024 runs", file=sys.stderr, flush=True)
    g5, f5 = W.shock_tube_2d(2048, 1024, gamma=gamma)
    runs = evaluate(g5, W.make_state(g5, f5, gamma))
    rho_plain = runs["plain"][0]
    out = {"workload": "2D viscous shock tube 2048x1024 (Re=200, FP64) from t=0 to t=1e-4; "
                       "network trained on theta^s of the 1000x500 tube after steps "
                       "1, 2, 3, 5, 10, 20, 50",
           "train": {"samples": int(Xt.shape[0]), "held_out": nhold, "steps": args.learned_train_steps,
                     "batch": 1024, "lr": 2e-3, "seconds": round(train_s, 2),
                     "loss_held_out_before": float(l0.item()),
                     "loss_held_out_after": float(l1.item()),
                     "fraction_theta_s_below_1": round(frac_lt1, 4),
                     "rmse_held_out_where_theta_s_below_1": round(rmse_low, 5),
                     "rmse_of_constant_1_there": round(rmse_one, 5)}}
    for name, (rho, n, ms) in runs.items():
        out[name] = {"value": g5.dof_sites * 3 * n / (ms / 1e3), "unit": "DOF-updates/s",
                     "steps": n, "ms": round(ms, 1),
                     "l1_rho_vs_plain": float(np.abs(rho - rho_plain).sum() * g5.dx * g5.dy)}
    # the same comparison at the training grid (1000 x 500, to the same t)
    runs3 = evaluate(g3, W.make_state(g3, f3, gamma))
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
