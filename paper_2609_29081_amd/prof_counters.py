"""HBM traffic and FP64 instruction counts of the fused 2D stage kernel
from rocprofv3 counters.

    python -m paper_2609_29081_amd.prof_counters [--mixed]            # driver (on the GPU host)
    python -m paper_2609_29081_amd.prof_counters --target [--mixed]   # profiled program
    python -m paper_2609_29081_amd.prof_counters --target-batch       # batched sweep
    python -m paper_2609_29081_amd.prof_counters --target-learned     # learned blend

The driver runs three counter passes (FETCH_SIZE; WRITE_SIZE; the FP64 and
LDS instruction counters) over the target, which launches the stage kernel on the 1000 x 500 shock tube (the
benchmark's launch configuration, averaged over the three RK3 stage kinds;
the same launch sequence as the roofline pass of bench.py)
and then a plain device copy of known size.  Each counter is scaled by what
it reads for that copy (bytes moved / counter value).  Executed FP64 flops
count 64 lanes per wave instruction (2 per FMA).  The driver writes
traffic.json and stage2d_shock_tube_1000x500_counters.md into its output
folder (--out); copied into profiles/, traffic.json is what bench.py reports
as the measured traffic and executed flops, as long as its hash of the
kernel sources still matches (a stale measurement is never reported).
With --mixed the same is done for the mixed-precision stage (FP32 stencils),
counting FP32 and FP64 instructions, into traffic_mixed.json and
stage2d_mixed_shock_tube_1000x500_counters.md.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 256 * 1024 * 1024
N1, N2 = 1000, 500


def stage_sequence(S, U0, reps: int) -> None:
    """reps x the three RK3 stage kinds from U0 at its CFL dt, each launch a
    complete stage (af_rk_stage never stops early); the launch sequence
    whose mean duration bench.py reports in its roofline"""
    import torch
    U1 = torch.empty_like(U0)
    U2 = torch.empty_like(U0)
    dt_dev = S.af_cfl_dt(U0)
    for _ in range(reps):
        S.af_rk_stage(0, None, U0, U1, dt_dev=dt_dev)
        S.af_rk_stage(1, U0, U1, U2, dt_dev=dt_dev)
        S.af_rk_stage(2, U0, U2, U1, dt_dev=dt_dev)


def workload(name: str, n1: int, n2: int):
    """(grid, initial data, physics keywords) of a profiled workload: the
    viscous shock tube (Re = 200) or the smooth vortex wave (n1 x n1)"""
    from paper_2609_29081_amd import workloads as W
    if name == "vortex":
        g, f = W.vortex_wave_2d(n1)
        return g, f, dict(mu=1e-3, Pr=0.72)
    g, f = W.shock_tube_2d(n1, n2)
    return g, f, dict(mu=0.005, Pr=0.73)


def target(reps: int = 10, mixed: bool = False, wl: str = "tube", n1: int = N1,
           n2: int = N2) -> None:
    sys.path.insert(0, ROOT)
    import torch

    from paper_2609_29081_amd import af
    from paper_2609_29081_amd import workloads as W

    g, f, phys = workload(wl, n1, n2)
    S = af.Solver(g, cfl_c=0.2, cfl_v=0.05, precision=af.PREC_MIXED if mixed else af.PREC_FP64,
                  **phys)
    U0 = S.to_device(W.make_state(g, f, 1.4))
    stage_sequence(S, U0, reps)
    torch.cuda.synchronize()
    a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print("target done", flush=True)


def target_batch(steps: int = 3) -> None:
    """the batched form's launches: the 64-instance shock-tube sweep (mixed
    precision), tuned, then `steps` accepted steps of every instance with
    HIP-graph replay (for a kernel trace of the batch stage kernel)"""
    sys.path.insert(0, ROOT)
    from paper_2609_29081_amd import af
    from paper_2609_29081_amd import workloads as W

    insts = W.shock_tube_sweep(64, seed=0)
    solvers = [af.Solver(g, precision=af.PREC_MIXED, cfl_c=0.2, cfl_v=0.05, **kw)
               for g, f, kw in insts]
    states = [S.to_device(W.make_state(g, f, kw["gamma"])) for S, (g, f, kw) in zip(solvers, insts)]
    B = af.Batch(solvers)
    B.af_batch_tune(states, 0.0, 1e30, reps=1)
    st, n, t, att = B.af_batch_run(states, 0.0, 1e30, steps, attempts_per_slot=4, use_graph=True)
    assert st == [af.AF_OK] * len(insts)
    print("target done: variant", af.stage_variants()[B.variant][0], "attempts", sum(att),
          flush=True)


def target_learned(steps: int = 3) -> None:
    """the learned form's launches: `steps` steps of the 2048 x 1024 shock
    tube (FP64) with the learned blend (seeded initial network: inference
    costs the same for any weights), for a kernel trace of the blend
    inference beside the stage kernel"""
    sys.path.insert(0, ROOT)
    import torch

    from paper_2609_29081_amd import af
    from paper_2609_29081_amd import workloads as W

    g, f = W.shock_tube_2d(2048, 1024)
    S = af.Solver(g, mu=0.005, Pr=0.73, cfl_c=0.2, cfl_v=0.05,
                  limiter=af.LIM_ALL | af.LIM_LEARNED)
    P = torch.as_tensor(W.mlp_init(0), device=S.device)
    S.af_set_blend_net(P)
    U = S.to_device(W.make_state(g, f, 1.4))
    st, n, t = S.af_run(U, 0.0, 1e30, steps, check_every=1)
    torch.cuda.synchronize()
    print("target done: status", st, "steps", n, flush=True)


FP64_COUNTERS = ["SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_ADD_F64",
                 "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VALU", "SQ_INSTS_LDS"]
MIXED_COUNTERS = ["SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_ADD_F32",
                  "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_ADD_F64",
                  "SQ_INSTS_VALU", "SQ_INSTS_LDS"]


def _target_args(mixed: bool, wl: str, n1: int, n2: int) -> list:
    return ["--target", "--workload", wl, "--n1", str(n1), "--n2", str(n2)] + \
        (["--mixed"] if mixed else [])


def _pass(counters: list, outdir: str, mixed: bool = False, wl: str = "tube", n1: int = N1,
          n2: int = N2) -> dict:
    """one rocprofv3 run collecting `counters`; returns
    {counter: {"stage": [per launch], "copy": [per launch]}}"""
    cmd = ["timeout", "-s", "KILL", "120", "rocprofv3", "--pmc", " ".join(counters),
           "--output-format", "csv", "-d", outdir, "-o", "run", "--", sys.executable, "-m",
           "paper_2609_29081_amd.prof_counters"] + _target_args(mixed, wl, n1, n2)
    env = dict(os.environ, TMPDIR="/tmp",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    subprocess.run(cmd, check=True, cwd="/tmp", env=env)
    files = glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True)
    vals = {c: {"stage": [], "copy": []} for c in counters}
    for fn in files:
        for r in csv.DictReader(open(fn)):
            name, cname = r["Kernel_Name"], r["Counter_Name"]
            if cname not in vals:
                continue
            v = float(r["Counter_Value"])
            if "k_stage" in name:
                vals[cname]["stage"].append(v)
            elif "copyBuffer" in name:
                vals[cname]["copy"].append(v)
    return vals


def driver(outroot: str, mixed: bool = False, wl: str = "tube", n1: int = N1,
           n2: int = N2) -> None:
    sys.path.insert(0, ROOT)
    import bench

    if wl == "vortex":
        n2 = n1
    res = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        res[c] = _pass([c], os.path.join(outroot, c.lower()), mixed, wl, n1, n2)[c]
    ilist = MIXED_COUNTERS if mixed else FP64_COUNTERS
    isa = _pass(ilist, os.path.join(outroot, "isa"), mixed, wl, n1, n2)
    per = {c: sum(isa[c]["stage"]) / len(isa[c]["stage"]) for c in ilist}
    flops = 64.0 * (2.0 * per["SQ_INSTS_VALU_FMA_F64"] + per["SQ_INSTS_VALU_MUL_F64"]
                    + per["SQ_INSTS_VALU_ADD_F64"])
    flops32 = (64.0 * (2.0 * per["SQ_INSTS_VALU_FMA_F32"] + per["SQ_INSTS_VALU_MUL_F32"]
                       + per["SQ_INSTS_VALU_ADD_F32"]) if mixed else 0.0)
    fetch_kib = sum(res["FETCH_SIZE"]["stage"]) / len(res["FETCH_SIZE"]["stage"])
    write_kib = sum(res["WRITE_SIZE"]["stage"]) / len(res["WRITE_SIZE"]["stage"])
    copy_fetch = max(res["FETCH_SIZE"]["copy"])
    copy_write = max(res["WRITE_SIZE"]["copy"])
    f_scale = COPY_BYTES / copy_fetch      # bytes per counter unit, reads
    w_scale = COPY_BYTES / copy_write      # bytes per counter unit, writes
    fetch_b = fetch_kib * f_scale
    write_b = write_kib * w_scale
    out = {"kernel": "stage2d", "precision": "mixed" if mixed else "fp64", "n1": n1, "n2": n2,
           "workload": wl,
           "kernel_source_hash": bench.kernel_source_hash(),
           "fetch_counter_kib": fetch_kib, "write_counter_kib": write_kib,
           "copy_fetch_counter": copy_fetch, "copy_write_counter": copy_write,
           "fetch_scale_bytes_per_unit": f_scale, "write_scale_bytes_per_unit": w_scale,
           "fetch_bytes": fetch_b, "write_bytes": write_b,
           "bytes_per_launch": fetch_b + write_b,
           "launches_averaged": len(res["FETCH_SIZE"]["stage"]),
           "instructions_per_launch": per,
           "fp64_flops_per_launch": flops,
           "fp32_flops_per_launch": flops32}
    prof = outroot
    os.makedirs(prof, exist_ok=True)
    tag = "_mixed" if mixed else ""
    wname = "shock_tube" if wl == "tube" else "vortex_wave"
    base = wl == "tube" and (n1, n2) == (N1, N2)
    jname = f"traffic{tag}.json" if base else f"traffic{tag}_{wname}_{n1}x{n2}.json"
    with open(os.path.join(prof, jname), "w") as fh:
        json.dump(out, fh, indent=1)
    cmdline = "python -m paper_2609_29081_amd.prof_counters" + (" --mixed" if mixed else "") + \
        ("" if base else f" --workload {wl} --n1 {n1} --n2 {n2}")
    g, _, _ = workload(wl, n1, n2)
    alg = 8.0 * 8.0 / 3.0 * g.state_len
    what = "mixed-precision (FP32 stencils, FP64 blends and updates)" if mixed else "FP64"
    md = [f"# Counters of the fused 2D stage kernel, {what} ({wname.replace('_', ' ')} {n1}x{n2})", "",
          f"Command: `{cmdline}` (three rocprofv3 passes, `--pmc FETCH_SIZE`,",
          f"`--pmc WRITE_SIZE`, `--pmc {' '.join(ilist)}`, each over",
          f"`python -m paper_2609_29081_amd.prof_counters {' '.join(_target_args(mixed, wl, n1, n2))}`: "
          "ten rounds of the three RK3 stage kinds (the sequence bench.py times for its roofline):",
          "complete stage launches at the CFL dt of the initial state, then a 256 MiB device copy",
          "for calibration).", "",
          "| quantity | value |", "|---|---|",
          f"| stage launches averaged | {out['launches_averaged']} |",
          f"| FETCH_SIZE per launch (counter, KiB) | {fetch_kib:.1f} |",
          f"| WRITE_SIZE per launch (counter, KiB) | {write_kib:.1f} |",
          f"| copy of {COPY_BYTES} B: FETCH_SIZE / WRITE_SIZE (counter) | {copy_fetch:.1f} / {copy_write:.1f} |",
          f"| scale, bytes per counter unit (read / write) | {f_scale:.1f} / {w_scale:.1f} |",
          f"| read bytes per launch | {fetch_b / 1e6:.1f} MB |",
          f"| written bytes per launch | {write_b / 1e6:.1f} MB |",
          f"| total per launch | {(fetch_b + write_b) / 1e6:.1f} MB |",
          "| algorithmic bytes per launch (mean of the 3 stages: 5/3 states read, 1 written) | "
          f"{alg / 1e6:.1f} MB |",
          f"| kernel source hash | {out['kernel_source_hash']} |"]
    md += ["", "| instruction counter (per launch, wave instructions) | value |", "|---|---|"]
    md += [f"| {c} | {per[c]:.4g} |" for c in ilist]
    md += [f"| executed FP64 flops per launch (64 lanes x (2 FMA + MUL + ADD)) | {flops:.4g} |"]
    if mixed:
        md += [f"| executed FP32 flops per launch (64 lanes x (2 FMA + MUL + ADD)) | {flops32:.4g} |"]
    name = f"stage2d{tag}_{wname}_{n1}x{n2}_counters.md"
    with open(os.path.join(prof, name), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print(json.dumps(out))


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--target", action="store_true")
    ap.add_argument("--mixed", action="store_true")
    ap.add_argument("--target-batch", action="store_true")
    ap.add_argument("--target-learned", action="store_true")
    ap.add_argument("--workload", choices=["tube", "vortex"], default="tube")
    ap.add_argument("--n1", type=int, default=N1)
    ap.add_argument("--n2", type=int, default=N2)
    ap.add_argument("--out", default=os.path.join(tempfile.gettempdir(), "af_counters"))
    a = ap.parse_args()
    if a.target_learned:
        target_learned()
    elif a.target_batch:
        target_batch()
    elif a.target:
        target(mixed=a.mixed, wl=a.workload, n1=a.n1, n2=a.n1 if a.workload == "vortex" else a.n2)
    else:
        driver(a.out, mixed=a.mixed, wl=a.workload, n1=a.n1, n2=a.n2)
