"""Benchmark: DG-apply DoF/s and time-to-U on one MI355X.

Workload: the thin-coating cylinder (2000 hexahedra at p = 6, 2,058,000 DoF;
coating 1e-3 R of 140 GPa / 0.23 on fused silica, 24 graded substrate
elements), synthetic seeded inputs resident in HBM.

A timed step is one pass of the hot path over the workload: the load vector,
the preconditioned Krylov solve (FP32 preconditioner inside FP64 FGMRES),
the layer energies and S_x.  The headline value is the DG-apply throughput
(FP64 operator applications per second times DoF), measured with HIP events
on the stream the kernels run on; the JSON line also carries the FP32 apply
rate, time-to-U of the FP64- and FP32-preconditioned solves, the roofline of
the dominant kernel and the oracle's CPU rate on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def interior_face_slots(spec):
    """Element faces with a neighbour (each read once by the neighbour's flux)."""
    n_z = sum(l["n_elem"] for l in spec["layers"])
    if spec["domain"] == "cylinder":
        m = 2 ** spec["refine"]
        n_cols = 5 * m * m
        boundary_edges = 4 * m
    else:
        n_cols = spec["nx"] * spec["ny"]
        boundary_edges = 2 * (spec["nx"] + spec["ny"])
    side = (4 * n_cols - boundary_edges) * n_z
    vert = 2 * n_cols * (n_z - 1)
    return side + vert, n_cols, n_z


def apply_bytes(spec, rbytes):
    """Algorithmic bytes of one launch of the volume-and-flux kernel: its own
    u, the neighbours' face tractions, the output, and the column geometry."""
    N = spec["p"] + 1
    E = W.n_elements(spec)
    slots, n_cols, n_z = interior_face_slots(spec)
    return rbytes * (6 * N ** 3 * E + 3 * N * N * slots + n_cols * (5 * N * N + 4 * N) + 2 * n_z) \
        + 4 * (8 * n_cols + n_z)


def traction_bytes(spec, rbytes):
    N = spec["p"] + 1
    E = W.n_elements(spec)
    _, n_cols, n_z = interior_face_slots(spec)
    return rbytes * (3 * N ** 3 * E + 18 * N * N * E + n_cols * 5 * N * N + n_z)


def apply_flops(spec):
    """Flops of one operator application (both passes): 18 sum-factorised
    contractions of 2N flops per node, plus the pointwise metric, lift,
    stress and flux work (about 160 flops per node)."""
    N = spec["p"] + 1
    E = W.n_elements(spec)
    return E * N ** 3 * (18 * 2 * N + 160)


def time_launches(fn, n, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(n):
        fn()
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / 1e3 / n


def cpu_baseline(spec, budget_s=15.0):
    """The oracle's operator application timed on the host on a bounded sample
    of the same workload (whole applications of A u)."""
    from oracle import dg
    O = dg.Problem(spec)
    u = W.random_field(spec, seed=0)
    t0 = time.perf_counter()
    n = 0
    while True:
        dg.apply(O, u)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = (time.perf_counter() - t0) / n
    return {"value": W.n_dof(spec) / dt, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} oracle applications of A u on the full {W.n_dof(spec)}-DoF workload "
                      f"(NumPy FP64, single thread), {dt:.2f} s each"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=50, help="operator applications per timed step")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only a plain 256 MiB device copy (HBM-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is described, not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2111_06893_amd as dgtn

    if args.calib_copy:
        a = torch.ones(32 * 2 ** 20, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": a.numel() * 8, "bytes_written": b.numel() * 8}))
        return

    spec = W.config2()
    n_dof = W.n_dof(spec)
    P = dgtn.Problem(spec)
    P.bind()
    stream = torch.cuda.current_stream()
    u64 = torch.from_numpy(W.random_field(spec, seed=0)).cuda()
    u32 = u64.float()
    o64 = torch.empty_like(u64)
    o32 = torch.empty_like(u32)

    def app64():
        P.apply(u64, o64)

    def app32():
        P.apply(u32, o32)

    for _ in range(args.warmup * args.reps):
        app64()
        app32()
    torch.cuda.synchronize()

    # timed steps: the full operator application, FP64 (headline) and FP32
    t64, t32 = [], []
    for _ in range(args.steps):
        t64.append(time_launches(app64, args.reps, stream))
        t32.append(time_launches(app32, args.reps, stream))
    torch.cuda.synchronize()
    a64 = float(np.median(t64))
    a32 = float(np.median(t32))

    # per-kernel durations for the roofline (same stream, HIP events)
    P.apply_stage(u64, o64, 1)
    k_apply64 = time_launches(lambda: P.apply_stage(u64, o64, 2), args.reps * 4, stream)
    k_trac64 = time_launches(lambda: P.apply_stage(u64, o64, 1), args.reps * 4, stream)
    P.apply_stage(u32, o32, 1)
    k_apply32 = time_launches(lambda: P.apply_stage(u32, o32, 2), args.reps * 4, stream)
    k_trac32 = time_launches(lambda: P.apply_stage(u32, o32, 1), args.reps * 4, stream)

    by64 = apply_bytes(spec, 8)
    fl = apply_flops(spec)
    out = {
        "metric": "DG-apply DoF/s; time-to-U at 1e-8 rel err, FP32-precond vs FP64 solve",
        "value": n_dof / a64,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": a64 * args.reps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "thin-coating cylinder, 2000 hex elements, p=6, 2,058,000 DoF "
                               "(coating 1e-3 R, 140 GPa/0.23 on 72 GPa/0.17, 24 graded substrate elements)",
                   "n_dof": n_dof, "elements": W.n_elements(spec), "p": spec["p"],
                   "applies_per_step": args.reps},
        "apply_fp64_us": a64 * 1e6,
        "apply_fp32_us": a32 * 1e6,
        "apply_fp32_dof_per_s": n_dof / a32,
        "kernels_us": {"k_traction_f64": k_trac64 * 1e6, "k_apply_f64": k_apply64 * 1e6,
                       "k_traction_f32": k_trac32 * 1e6, "k_apply_f32": k_apply32 * 1e6},
        "roofline": {"bound": "hbm", "kernel": "k_apply<7,double>", "achieved": by64 / k_apply64 / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": by64 / k_apply64 / 1e9 / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": by64},
        "roofline_f32": {"bound": "hbm", "kernel": "k_apply<7,float>",
                         "achieved": apply_bytes(spec, 4) / k_apply32 / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": apply_bytes(spec, 4) / k_apply32 / 1e9 / HBM_PEAK_GBS},
        "flop_frac_f64": fl / a64 / 1e12 / FP64_PEAK_TFLOPS,
        "flop_frac_f32": fl / a32 / 1e12 / FP32_PEAK_TFLOPS,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
