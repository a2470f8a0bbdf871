"""Benchmark: DG-apply DoF/s and time-to-U on one MI355X.

Headline workload: the forty-layer crystalline coating (forty alternating
cubic-crystal layers of 1e-5 R, (119, 53.8, 59.5) and (120, 57, 58.9) GPa, on a
fused-silica substrate of 60 graded elements; 80 columns x 100 z-elements =
8000 hexahedra at p = 5, 5,184,000 DoF), the largest of the benchmark
workloads; synthetic seeded inputs resident in HBM.

One timed step is one pass of the whole hot path over that workload: the load
vector; a block of FP64 operator applications (the DG apply, timed with HIP
events on the stream it runs on); the FP32-preconditioned flexible-CG solve at
the stopping tolerance calibrated for a 1e-8 error in the layer energies; the
layer energies and the compliance 1/2 u.b; S_x (one loss angle per layer); and
the adjoint gradient of S_x with respect to the forty coating thicknesses and
the six cubic constants (one more solve and the parameter derivatives).  The
headline value is the FP64 DG-apply throughput (DoF x applications / s) of the
apply blocks inside the timed steps.

Beside it, untimed records: the FP32 apply rate and the per-kernel rooflines;
time-to-U of the FP64- and FP32-preconditioned solves; the thin-coating
cylinder (2000 elements, p = 6, 2,058,000 DoF) with its own apply rates and
time-to-U; the apply on the thin-coating mesh refined once and twice across the
disk (8,232,000 and 32,928,000 DoF: working sets beyond the 256 MB
Infinity Cache, where the operator streams from HBM); the seeded-beam-width
cylinders (seeds 0-9) against the oracle's energies with time-to-U of both
preconditioners; the design loop and adaptive refinement; and the oracle timed
on the host cores (all cores, one oracle process per core).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3

HEADLINE = "forty_layer"


def workload(name):
    """Problem description of a named benchmark workload."""
    if name == "forty_layer":
        return W.config5(p=5)
    if name == "forty_layer_p6":
        return W.config5(p=6)
    if name == "thin_coating":
        return W.config2()
    if name in ("thin_coating_r3", "thin_coating_r4"):
        s = W.config2()
        s["refine"] = int(name[-1])
        return s
    raise ValueError(name)


WORKLOAD_TEXT = {
    "forty_layer": "forty 1e-5 R cubic-crystal layers on fused silica, 80 columns x (40 + 60 graded) "
                   "= 8000 hex elements, p=5, 5,184,000 DoF",
    "forty_layer_p6": "the forty-layer coating at p=6, 8000 hex elements, 8,232,000 DoF",
    "thin_coating": "thin-coating cylinder, 2000 hex elements, p=6, 2,058,000 DoF (coating 1e-3 R, "
                    "140 GPa/0.23 on 72 GPa/0.17, 24 graded substrate elements)",
    "thin_coating_r3": "thin-coating mesh refined once across the disk: 320 columns x 25 = 8000 hex "
                       "elements, p=6, 8,232,000 DoF",
    "thin_coating_r4": "thin-coating mesh refined twice across the disk: 1280 columns x 25 = 32000 hex "
                       "elements, p=6, 32,928,000 DoF",
}

# The rocprofv3 runs whose output --summarize reads (from the repository root).
PROFILED = ("forty_layer", "thin_coating", "thin_coating_r4")


def profile_commands():
    c = {}
    for w in PROFILED:
        c[f"trace_{w}"] = (f"rocprofv3 --kernel-trace --stats -d prof_out/trace_{w} -o run --output-format csv -- "
                           f"python3 bench.py --apply-only {w} --steps 2 --reps 20")
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            c[f"{ctr.split('_')[0].lower()}_{w}"] = (
                f"rocprofv3 --pmc {ctr} -d prof_out/{ctr.split('_')[0].lower()}_{w} -o run --output-format csv -- "
                f"python3 bench.py --apply-only {w} --steps 1 --reps 4")
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        k = ctr.split('_')[0].lower()
        c[f"{k}_copy"] = (f"rocprofv3 --pmc {ctr} -d prof_out/{k}_copy -o run --output-format csv -- "
                          "python3 bench.py --calib-copy")
    for n in (1, 4):
        c[f"solve_{n}"] = (f"rocprofv3 --kernel-trace --stats -d prof_out/solve_{n} -o run --output-format csv -- "
                           f"python3 bench.py --one-solve {HEADLINE} --passes {n}")
    return c


# The paper's own wall times of its CPU solver (Sec. 3 and Sec. 4), quoted with their
# hardware as context: other configurations and machines, not a target.
PAPER_CPU_TIMINGS = {
    "hardware": "Intel Haswell E5-2630v3 2.4 GHz, 16-core nodes, 15 cores used per node",
    "single coating, sub-percent error in U": "30 s on 15 cores",
    "single coating, fractional error 1e-5": "about 2 min wall (half a core-hour) on 15 cores",
    "simple configurations": "seconds to minutes on 15 cores",
    "nine sub-micron crystalline layers": "about 1 hour on 45 cores",
}


# ---------------------------------------------------------------------------
# byte and flop models of the operator kernels

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
    """Algorithmic bytes of one launch of the face-traction kernel: u in,
    tractions on the six faces out, the column geometry."""
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


def time_isolated(fn, n, stream):
    """Average duration of single launches, each bracketed by its own pair of
    HIP events on the launch stream (what a per-dispatch trace reports; the
    block average of time_launches also lets a kernel's tail overlap the next
    launch's start)."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    evs[-1][1].synchronize()
    return sum(a.elapsed_time(b) for a, b in evs) / n / 1e3


def kernel_name(spec, kind, prec):
    return f"k_{kind}<{spec['p'] + 1},{'double' if prec == 64 else 'float'}>"


def apply_record(name, P, reps, rounds, stream):
    """Apply rates (whole apply, FP64 and FP32) and per-kernel rooflines of a
    bound problem; HIP-event averages over `rounds` blocks of `reps` launches,
    medians over the blocks."""
    import torch
    spec = P.spec
    n_dof = W.n_dof(spec)
    u64 = torch.from_numpy(W.random_field(spec, seed=0)).cuda()
    u32 = u64.float()
    o64, o32 = torch.empty_like(u64), torch.empty_like(u32)
    P.apply(u64, o64)
    P.apply(u32, o32)
    t = {}
    for prec, u, o in ((64, u64, o64), (32, u32, o32)):
        t[f"apply{prec}"] = float(np.median([time_launches(lambda: P.apply(u, o), reps, stream)
                                             for _ in range(rounds)]))
        P.apply_stage(u, o, 1)
        t[f"k_apply{prec}"] = float(np.median([time_launches(lambda: P.apply_stage(u, o, 2), reps, stream)
                                               for _ in range(rounds)]))
        t[f"k_traction{prec}"] = float(np.median([time_launches(lambda: P.apply_stage(u, o, 1), reps, stream)
                                                  for _ in range(rounds)]))
        P.apply_stage(u, o, 1)
        t[f"k_apply{prec}_iso"] = time_isolated(lambda: P.apply_stage(u, o, 2), reps, stream)
        t[f"k_traction{prec}_iso"] = time_isolated(lambda: P.apply_stage(u, o, 1), reps, stream)
    rec = {"workload": WORKLOAD_TEXT[name], "n_dof": n_dof, "elements": W.n_elements(spec), "p": spec["p"],
           "apply_fp64_us": t["apply64"] * 1e6, "apply_fp32_us": t["apply32"] * 1e6,
           "apply_fp64_dof_per_s": n_dof / t["apply64"], "apply_fp32_dof_per_s": n_dof / t["apply32"],
           "kernels_us": {f"k_{k}_f{p}": t[f"k_{k}{p}"] * 1e6 for k in ("traction", "apply") for p in (64, 32)},
           "kernels_isolated_launch_us": {f"k_{k}_f{p}": t[f"k_{k}{p}_iso"] * 1e6 for k in ("traction", "apply")
                                          for p in (64, 32)},
           "flop_frac_f64": apply_flops(spec) / t["apply64"] / 1e12 / FP64_PEAK_TFLOPS,
           "flop_frac_f32": apply_flops(spec) / t["apply32"] / 1e12 / FP32_PEAK_TFLOPS,
           "working_set_fp64_MB": (2 * 8 * n_dof + 8 * 18 * (spec["p"] + 1) ** 2 * W.n_elements(spec)) / 1e6}
    for kind, fn in (("apply", apply_bytes), ("traction", traction_bytes)):
        for prec in (64, 32):
            by = fn(spec, prec // 8)
            ach = by / t[f"k_{kind}{prec}"] / 1e9
            rec[f"roofline_{kind}_f{prec}"] = {
                "bound": "hbm", "kernel": kernel_name(spec, kind, prec), "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "bytes_per_launch": by,
                "traffic": measured_traffic(name, kind) if prec == 64 else None}
    rec["apply_pair_hbm_frac_f64"] = (apply_bytes(spec, 8) + traction_bytes(spec, 8)) / t["apply64"] / 1e9 \
        / HBM_PEAK_GBS
    return rec


# ---------------------------------------------------------------------------
# solves

def time_to_u(P, target=1e-8, log=None, rtols=(1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10), ref_max_iter=200):
    """Time-to-U of the FP64- and the FP32-preconditioned solve.

    The reference U is a tight FP64 solve in the same run, stopped at the
    workload's FP64 residual floor (reported as stagnation).  For each
    preconditioner precision the loosest stopping tolerance whose layer
    energies lie within `target` of the reference is found by a sweep, then a
    solve at that tolerance is timed from the call to the energies on the host
    (load vector and geometry already resident), median of three."""
    import torch
    import paper_2111_06893_amd as dgtn

    def solve(prec, rtol, max_iter=40000):
        opts = dgtn.default_opts(prec, rtol=rtol, max_iter=max_iter)
        b = P.rhs()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, st = P.solve(b, opts=opts, raise_on_noconv=False)
        U = P.energy(u)
        dt = time.perf_counter() - t0
        return U, st, dt

    Uref, st, dt = solve(64, 1e-12, max_iter=ref_max_iter)
    if log:
        log(f"reference solve: {st.iters} iterations, rel.res {st.rel_res:.2e}, {dt:.2f} s")
    out = {"reference": {"U": float(Uref.sum()), "iters": st.iters, "rel_res": st.rel_res, "seconds": dt}}
    for prec in (64, 32):
        chosen = None
        for rtol in rtols:
            U, st, dt = solve(prec, rtol)
            err = float(np.max(np.abs(U - Uref) / np.abs(Uref)))
            if log:
                log(f"precond fp{prec} rtol {rtol:.0e}: {st.iters} it, {dt:.3f} s, max layer U err {err:.2e}")
            if err <= target:
                chosen = rtol
                break
        if chosen is None:
            out[f"fp{prec}_precond"] = None
            continue
        runs = [solve(prec, chosen) for _ in range(3)]
        U, st, dt = sorted(runs, key=lambda r: r[2])[1]
        err = float(np.max(np.abs(U - Uref) / np.abs(Uref)))
        out[f"fp{prec}_precond"] = {"time_to_U_s": dt, "iters": st.iters, "rtol": chosen,
                                    "U_rel_err": err, "ms_per_iter": dt / max(st.iters, 1) * 1e3}
    t64 = (out.get("fp64_precond") or {}).get("time_to_U_s")
    t32 = (out.get("fp32_precond") or {}).get("time_to_U_s")
    if t64 and t32:
        out["speedup_fp32_precond"] = t64 / t32
    return out


def seeded_beams(log, seeds=range(10)):
    """The cylinder of 40 elements at p = 5 with the beam width r0 drawn from
    U[0.05, 0.2] R per seed: for each preconditioner precision, time-to-U
    against the oracle's converged energy (the loosest stopping tolerance whose
    total energy lies within 1e-8 of the oracle's, timed, median of three) and
    the energy error of a tight solve."""
    import torch
    import paper_2111_06893_amd as dgtn
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "energies.json")))
    rows = []
    for s in seeds:
        g = gold.get(f"config3_seed{s}")
        if g is None:
            continue
        spec = W.config3(seed=s)
        P = dgtn.Problem(spec)
        Uo = g["U"]
        row = {"seed": s, "r0": spec["load"]["r0"]}
        for prec in (64, 32):
            def solve(rtol):
                o = dgtn.default_opts(prec, rtol=rtol, max_iter=20000)
                b = P.rhs()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                u, st = P.solve(b, opts=o, raise_on_noconv=False)
                U = P.energy(u).sum()
                return abs(U / Uo - 1), time.perf_counter() - t0, st.iters
            solve(1e-11)   # binds the hierarchy of this precision (not timed)
            err_tight, _, _ = solve(1e-11)
            row[f"fp{prec}_U_err_tight"] = err_tight
            for rtol in (1e-6, 1e-7, 1e-8, 1e-9, 1e-10, 1e-11):
                e, _, _ = solve(rtol)
                if e <= 1e-8:
                    runs = sorted(solve(rtol) for _ in range(3))
                    row[f"fp{prec}"] = {"rtol": rtol, "U_err": runs[1][0], "time_to_U_s": sorted(r[1] for r in runs)[1],
                                        "iters": runs[1][2]}
                    break
        P.close()
        rows.append(row)
    errs = {p: [r[f"fp{p}_U_err_tight"] for r in rows] for p in (64, 32)}
    tt = {p: [r[f"fp{p}"]["time_to_U_s"] for r in rows if r.get(f"fp{p}")] for p in (64, 32)}
    out = {"workload": "cylinder R = H = 1, 40 hex elements, p=5, 25,920 DoF, beam width r0 ~ U[0.05, 0.2] R "
                       "per seed (numpy default_rng)",
           "seeds": rows,
           "U_err_vs_oracle_tight": {f"fp{p}_precond": {"max": float(np.max(errs[p])), "median": float(np.median(errs[p]))}
                                     for p in (64, 32) if errs[p]},
           "time_to_U_median_s": {f"fp{p}_precond": float(np.median(tt[p])) for p in (64, 32) if tt[p]}}
    log(f"seeded beams: {len(rows)} seeds, tight-solve U error max {out['U_err_vs_oracle_tight']}, "
        f"time-to-U medians {out['time_to_U_median_s']}")
    return out


# ---------------------------------------------------------------------------
# the oracle on the host cores

def _cpu_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def _worker_env():
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    env["HIP_VISIBLE_DEVICES"] = ""      # the oracle processes never touch the GPU
    return env


def cpu_worker(name, budget_s):
    """One oracle process: whole applications of A u on the named workload for
    about budget_s seconds (setup not timed); prints its count and time."""
    from oracle import dg
    spec = workload(name)
    O = dg.Problem(spec)
    u = W.random_field(spec, seed=0)
    dg.apply(O, u)
    t0 = time.perf_counter()
    n = 0
    while True:
        dg.apply(O, u)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    print(json.dumps({"applies": n, "seconds": time.perf_counter() - t0}), flush=True)


def cpu_ttu_worker():
    """The oracle's own solve of the cylinder of 40 elements at p = 5 (block-
    Jacobi preconditioned CG, single thread) to a relative residual of 1e-10,
    with its energy error against the converged golden value."""
    from oracle import dg, solve
    spec = W.config1()
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "energies.json")))["config1"]["U"]
    t0 = time.perf_counter()
    O = dg.Problem(spec)
    b = dg.rhs(O)
    u, it, rel = solve.pcg(O, b, rtol=1e-10, maxit=60000)
    U = float(dg.energy_layers(O, u).sum())
    print(json.dumps({"seconds": time.perf_counter() - t0, "iters": it, "rel_res": rel,
                      "U_rel_err": abs(U / gold - 1)}), flush=True)


def start_cpu_ttu():
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-ttu-worker"], stdout=subprocess.PIPE,
                            stderr=subprocess.DEVNULL, env=_worker_env(), cwd=ROOT, text=True)


def cpu_baseline(name, budget_s, ttu_proc, log):
    """The oracle timed on the host cores: one single-threaded oracle process
    per core (at most 16), each applying A u on the full workload; the value is
    their summed throughput.  Also the oracle's time-to-U on the 40-element
    cylinder (run in a process of its own while the GPU work ran)."""
    info = _cpu_info()
    cores = max(1, min(info["affinity"], 16))
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", name, str(budget_s)],
                              stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, env=_worker_env(), cwd=ROOT,
                              text=True) for _ in range(cores)]
    res = []
    for p in procs:
        out, _ = p.communicate()
        res.append(json.loads(out.strip().splitlines()[-1]))
    n_dof = W.n_dof(workload(name))
    rates = [r["applies"] * n_dof / r["seconds"] for r in res]
    rec = {"value": float(np.sum(rates)), "unit": "DoF/s", "cores": cores, "kind": "oracle",
           "sample": f"{sum(r['applies'] for r in res)} oracle applications of A u on the full {n_dof}-DoF "
                     f"headline workload by {cores} single-threaded oracle processes (NumPy FP64) in parallel, "
                     f"~{budget_s:.0f} s each; {np.mean([r['seconds'] / r['applies'] for r in res]):.2f} s "
                     "per application per process",
           "per_core_dof_per_s": float(np.mean(rates)), **info}
    if ttu_proc is not None:
        out, _ = ttu_proc.communicate()
        try:
            t = json.loads(out.strip().splitlines()[-1])
            rec["time_to_U_cylinder_40el"] = {**t, "cores": 1,
                                             "method": "oracle CG with exact element-block inverses, rtol 1e-10",
                                             "workload": "cylinder R = H = 1, 40 hex elements, p=5, 25,920 DoF"}
        except (ValueError, IndexError):
            rec["time_to_U_cylinder_40el"] = None
    log(f"cpu baseline: {rec['value']:.3e} DoF/s on {cores} cores ({info['cpu_model']})")
    return rec


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=50, help="operator applications per timed step")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the untimed secondary records")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--apply-only", metavar="WORKLOAD",
                    help="operator applications only on a named workload (profiling runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only a plain 256 MiB device copy (HBM-counter calibration)")
    ap.add_argument("--one-solve", metavar="WORKLOAD",
                    help="setup and `passes` solve passes (solve + energies + adjoint) without applies")
    ap.add_argument("--passes", type=int, default=1)
    ap.add_argument("--summarize", metavar="PROF_DIR",
                    help="write profiles/ summaries from rocprofv3 output in PROF_DIR and exit")
    ap.add_argument("--cpu-worker", nargs=2, metavar=("WORKLOAD", "SECONDS"), help=argparse.SUPPRESS)
    ap.add_argument("--cpu-ttu-worker", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args.cpu_worker[0], float(args.cpu_worker[1]))
        return
    if args.cpu_ttu_worker:
        cpu_ttu_worker()
        return
    if args.summarize:
        summarize_profiles(args.summarize)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is described, not built.", file=sys.stderr)
        sys.exit(2)

    log = lambda m: print("[bench] " + m, file=sys.stderr, flush=True)  # noqa: E731
    ttu_proc = None if (args.no_cpu or args.apply_only or args.one_solve or args.calib_copy) else start_cpu_ttu()

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
    if args.apply_only:
        P = dgtn.Problem(workload(args.apply_only))
        P.bind()
        rec = apply_record(args.apply_only, P, args.reps, max(1, args.steps), torch.cuda.current_stream())
        print(json.dumps(rec))
        return
    if args.one_solve:
        one_solve(args.one_solve, args.passes)
        return

    spec = workload(HEADLINE)
    n_dof = W.n_dof(spec)
    n_coat = len(spec["layers"]) - 1
    t0 = time.perf_counter()
    P = dgtn.Problem(spec)
    P.bind(dgtn.default_opts(32))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    u64 = torch.from_numpy(W.random_field(spec, seed=0)).cuda()
    o64 = torch.empty_like(u64)

    def app64():
        P.apply(u64, o64)

    # calibration of the stopping tolerances (untimed): time-to-U of both preconditioners
    ttu = time_to_u(P, log=log)
    rtol32 = ttu["fp32_precond"]["rtol"] if ttu.get("fp32_precond") else 5e-8
    opts32 = dgtn.default_opts(32, rtol=rtol32, max_iter=20000)
    grad_params = [("thickness", k) for k in range(n_coat)] + [(c, m) for m in (1, 2) for c in ("c11", "c12", "c44")]
    T_K, f_Hz = 300.0, 100.0
    phi = np.r_[np.full(n_coat, 4e-4), 1e-7]          # synthetic loss angles: coating layers, substrate
    w_sx = 4 * 1.380649e-23 * T_K * phi / (np.pi * f_Hz * spec["load"]["F0"] ** 2)

    def step():
        """One pass of the hot path; returns (apply block seconds, breakdown)."""
        b = P.rhs()
        t_app = time_launches(app64, args.reps, stream)
        t0 = time.perf_counter()
        u, st = P.solve(b, opts=opts32, raise_on_noconv=False)
        U, comp = P.energy(u, compliance=True)
        sx = P.noise(U, phi, T_K, f_Hz)
        t1 = time.perf_counter()
        lam, st2 = P.solve(P.energy_grad(u, w_sx), opts=opts32, raise_on_noconv=False)
        g = P.grad(u, lam, grad_params, w_sx)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t_app, {"U_layers": U, "U_compl": comp, "S_x": sx, "dSx": g, "solve_iters": st.iters,
                       "adjoint_iters": st2.iters, "solve_s": t1 - t0, "adjoint_s": t2 - t1}

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_steps, t_apps, recs = [], [], []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_app, rec = step()
        torch.cuda.synchronize()
        t_steps.append(time.perf_counter() - t0)
        t_apps.append(t_app)
        recs.append(rec)
    a64 = float(np.median(t_apps))
    kern = apply_record(HEADLINE, P, args.reps, 5, stream)
    last = recs[-1]
    U = last["U_layers"]
    out = {
        "metric": "DG-apply DoF/s; time-to-U at 1e-8 rel err, FP32-precond vs FP64 solve",
        "value": n_dof / a64,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean(t_steps)) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[HEADLINE], "n_dof": n_dof, "elements": W.n_elements(spec),
                   "p": spec["p"], "applies_per_step": args.reps,
                   "precond": "fp32 multigrid V-cycle (p- then h-coarsening, then fiducial merged-layer levels) "
                              "with weighted overlapping column-Schwarz smoother (overlap 1, damping 0.65), "
                              "dense coarsest solve",
                   "solve_rtol": rtol32},
        "step": {"apply_block_ms": a64 * args.reps * 1e3,
                 "solve_ms": float(np.median([r["solve_s"] for r in recs])) * 1e3,
                 "adjoint_and_gradient_ms": float(np.median([r["adjoint_s"] for r in recs])) * 1e3,
                 "solve_iters": last["solve_iters"], "adjoint_iters": last["adjoint_iters"],
                 "U_coat": float(np.sum(U[:n_coat])), "U_sub": float(U[n_coat]), "U_compl": last["U_compl"],
                 "S_x": last["S_x"], "n_params": len(grad_params),
                 "dSx_dthickness_first_last": [float(last["dSx"][0]), float(last["dSx"][n_coat - 1])],
                 "dSx_dcubic": [float(x) for x in last["dSx"][n_coat:]],
                 "theta": "40 coating thicknesses, then (c11, c12, c44) of the two crystals"},
        "setup_s": setup_s,
        "apply_fp64_us": a64 * 1e6,
        "apply_fp32_us": kern["apply_fp32_us"],
        "apply_fp32_dof_per_s": kern["apply_fp32_dof_per_s"],
        "kernels_us": kern["kernels_us"],
        "roofline": kern["roofline_apply_f64"],
        "roofline_f32": kern["roofline_apply_f32"],
        "roofline_traction": kern["roofline_traction_f64"],
        "apply_pair_hbm_frac": kern["apply_pair_hbm_frac_f64"],
        "flop_frac_f64": kern["flop_frac_f64"],
        "flop_frac_f32": kern["flop_frac_f32"],
        "working_set_fp64_MB": kern["working_set_fp64_MB"],
        "time_to_U": ttu,
    }
    del P, u64, o64
    torch.cuda.empty_cache()
    if not args.no_extra:
        out["thin_coating"] = secondary("thin_coating", log, args.reps)
        out["forty_layer_p6"] = secondary("forty_layer_p6", log, args.reps)
        out["hbm_sweep"] = hbm_sweep(log, args.reps)
        out["seeded_beams"] = seeded_beams(log)
        out["design_loop"] = design_loop(log)
        out["design_mirror"] = design_mirror(log)
        out["adaptive_refinement"] = adaptive_refinement(log)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(HEADLINE, args.cpu_budget, ttu_proc, log)
    out["paper_cpu_timings"] = PAPER_CPU_TIMINGS
    print(json.dumps(out), flush=True)


def secondary(name, log, reps):
    """A secondary workload (the thin-coating cylinder, the forty-layer coating
    at p = 6): apply rates, kernel rooflines and time-to-U."""
    import torch
    import paper_2111_06893_amd as dgtn
    P = dgtn.Problem(workload(name))
    P.bind(dgtn.default_opts(32))
    rec = apply_record(name, P, reps, 5, torch.cuda.current_stream())
    rec["time_to_U"] = time_to_u(P, log=log)
    P.close()
    torch.cuda.empty_cache()
    log(f"{name}: apply {rec['apply_fp64_dof_per_s']:.3e} DoF/s")
    return rec


def hbm_sweep(log, reps):
    """The operator on the thin-coating mesh at 2.06M, 8.23M and 32.9M DoF: the
    larger two keep u, A u and the face tractions (0.3 and 1.1 GB in FP64)
    beyond the 256 MB Infinity Cache, so their applies stream from HBM."""
    import torch
    import paper_2111_06893_amd as dgtn
    rows = {}
    for name in ("thin_coating", "thin_coating_r3", "thin_coating_r4"):
        P = dgtn.Problem(workload(name))
        P.bind()
        rows[name] = apply_record(name, P, reps, 5, torch.cuda.current_stream())
        P.close()
        torch.cuda.empty_cache()
        log(f"hbm sweep {name}: {rows[name]['apply_fp64_dof_per_s']:.3e} DoF/s, k_apply frac "
            f"{rows[name]['roofline_apply_f64']['frac']:.3f}")
    return rows


def one_solve(name, passes):
    """Setup, then `passes` passes of: FP32-preconditioned solve at 5e-8,
    energies, adjoint solve and the coating-thickness derivatives (profiling:
    the difference of two runs with different pass counts is the solve loop
    alone, setup excluded)."""
    import torch
    import paper_2111_06893_amd as dgtn
    spec = workload(name)
    P = dgtn.Problem(spec)
    o = dgtn.default_opts(32, rtol=5e-8, max_iter=2000)
    P.bind(o)
    n = len(spec["layers"])
    w = np.r_[np.ones(n - 1), 0.0]
    params = [("thickness", k) for k in range(n - 1)]
    res = {}
    for _ in range(passes):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, st = P.solve(opts=o, raise_on_noconv=False)
        U = P.energy(u)
        lam, st2 = P.solve(P.energy_grad(u, w), opts=o, raise_on_noconv=False)
        g = P.grad(u, lam, params, w)
        torch.cuda.synchronize()
        res = {"seconds": time.perf_counter() - t0, "solve_iters": st.iters, "adjoint_iters": st2.iters,
               "U_coat": float(np.dot(w, U)), "dUcoat_first": float(g[0])}
    print(json.dumps(res))


def design_loop(log):
    """Untimed record of the gradient-driven design loop: the beam centre on the
    five-block cylinder (40 elements, p = 5) that minimises S_x on the line
    xc - yc = 0.2 (symmetry puts the optimum at (0.1, -0.1)); every evaluation is
    a forward solve, an adjoint solve and the beam derivatives."""
    import torch
    from paper_2111_06893_amd import design
    spec = W.config1()
    spec["load"] = {"F0": 1.0, "r0": 0.2, "xc": 0.25, "yc": 0.05}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = design.optimize(spec, [("xc", 0), ("yc", 0)], design.NoiseObjective([1e-4, 1e-4], 300.0, 100.0),
                        constraints=[design.fixed_sum([0, 1], 0.2, [1.0, -1.0])],
                        bounds=[(-0.6, 0.6), (-0.6, 0.6)], tol=1e-14, maxiter=40)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"design loop: beam centre {r.x.tolist()} after {r.n_evals} evaluations, {dt:.2f} s")
    return {"workload": "beam centre on xc - yc = 0.2 minimising S_x, five-block cylinder, 40 elements, p=5",
            "x": r.x.tolist(), "expected": [0.1, -0.1], "evaluations": r.n_evals, "seconds": dt,
            "S_x": r.fun}


def design_mirror(log, maxiter=30):
    """Untimed record of the design loop on the forty-layer mirror: S_x (loss
    angles 1e-4 on crystal A, 1e-5 on crystal B, 1e-7 on the substrate:
    synthetic) minimised over the forty coating thicknesses, with their sum held
    at its nominal 4e-4 R and each within [0.5, 1.5] of its nominal 1e-5 R.  A
    coating layer's energy is close to proportional to its thickness, so the
    problem is close to a linear programme, whose optimum puts the layers of
    lower phi times energy per thickness at the upper bound and the others at
    the lower.  Every evaluation is a mesh and hierarchy set-up, a forward and
    an adjoint solve and the forty thickness derivatives."""
    import torch
    import paper_2111_06893_amd as dgtn
    from paper_2111_06893_amd import design
    spec = workload(HEADLINE)
    n = len(spec["layers"]) - 1
    phi = np.r_[[1e-4 if spec["layers"][k]["material"] == 1 else 1e-5 for k in range(n)], 1e-7]
    d0 = np.array([spec["layers"][k]["thickness"] for k in range(n)])
    opts = dgtn.default_opts(32, rtol=5e-8, max_iter=2000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = design.optimize(spec, [("thickness", k) for k in range(n)], design.NoiseObjective(phi, 300.0, 100.0),
                        constraints=[design.fixed_sum(range(n), float(d0.sum()))],
                        bounds=[(0.5 * d, 1.5 * d) for d in d0], tol=1e-9, maxiter=maxiter,
                        engine=design.device_engine(opts, max_rel_res=1e-6))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ratio = r.x / d0
    low_phi = np.array([phi[k] < 1e-4 for k in range(n)])
    S0 = r.history[0][1]
    log(f"mirror design: S_x {S0:.4e} -> {r.fun:.4e} in {r.n_evals} evaluations, {dt:.1f} s")
    return {"workload": "forty-layer mirror: S_x over the forty coating thicknesses at fixed total thickness, "
                        "each in [0.5, 1.5] x 1e-5 R; loss angles 1e-4 (crystal A), 1e-5 (crystal B), 1e-7 "
                        "(substrate), synthetic",
            "S_x_start": S0, "S_x_end": r.fun, "evaluations": r.n_evals, "seconds": dt,
            "success": r.success, "message": r.message,
            "thickness_ratio_low_phi_layers": [float(ratio[low_phi].min()), float(ratio[low_phi].max())],
            "thickness_ratio_high_phi_layers": [float(ratio[~low_phi].min()), float(ratio[~low_phi].max())],
            "total_thickness_rel_change": float(r.x.sum() / d0.sum() - 1.0)}


def adaptive_refinement(log, steps=3):
    """Untimed record of adaptive refinement across the layers: the coated
    cylinder (coating 1e-3 R and substrate, one element each across their
    thickness, 20 columns, p = 3) through `steps` solve / z-face indicator /
    mark / refine steps."""
    import torch
    import paper_2111_06893_amd as dgtn
    from paper_2111_06893_amd import adapt
    spec = W.config4()
    spec["p"] = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec = adapt.adapt(spec, steps=steps, theta=0.6, opts=dgtn.default_opts(32, rtol=1e-9, max_iter=5000))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = [{"n_elem_per_layer": [l["n_elem"] for l in r.spec["layers"]], "n_dof": r.n_dof,
            "U_layers": r.U.tolist(), "eta_z_layers": r.eta_layers.tolist(), "marked": r.marked,
            "iters": r.iters, "rel_res": r.rel_res} for r in rec]
    log(f"adaptive refinement: {[o['n_elem_per_layer'] for o in out]}, {dt:.2f} s")
    return {"workload": "coated cylinder (coating 1e-3 R, 20 columns, p=3), refinement across the layers",
            "steps": out, "seconds": dt}


# ---------------------------------------------------------------------------
# profiles

def _short(name):
    return name.replace("dgtn::(anonymous namespace)::", "").replace("void ", "").split("(")[0][:72]


def summarize_profiles(prof_dir):
    """Writes profiles/ summaries from the rocprofv3 output under prof_dir (the
    runs of profile_commands()): kernel statistics of each apply-only trace,
    the HBM traffic of the operator kernels from FETCH_SIZE / WRITE_SIZE runs
    scaled by the same counters on a plain 256 MiB copy, and the kernels of the
    solve loop with setup excluded (the difference of a four-pass and a
    one-pass run)."""
    import collections
    import csv

    commands = profile_commands()
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)

    def rows(sub, fname):
        path = os.path.join(prof_dir, sub, fname)
        return list(csv.DictReader(open(path))) if os.path.exists(path) else None

    def pmc(sub, counter):
        agg = collections.defaultdict(list)
        for r in rows(sub, "run_counter_collection.csv") or []:
            if r["Counter_Name"] == counter:
                agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return agg

    copy_bytes = 32 * 2 ** 20 * 8
    cf = [v for k, vs in pmc("fetch_copy", "FETCH_SIZE").items() if "elementwise" in k for v in vs]
    cw = [v for k, vs in pmc("write_copy", "WRITE_SIZE").items() if "elementwise" in k for v in vs]
    fetch_factor = copy_bytes / (max(cf) * 1024.0) if cf else None
    write_factor = copy_bytes / (max(cw) * 1024.0) if cw else None
    printed = []
    for w in PROFILED:
        spec = workload(w)
        st = rows(f"trace_{w}", "run_kernel_stats.csv")
        if st:
            lines = [f"# Kernel durations, {WORKLOAD_TEXT[w]}", "", "Command (from the repository root, TMPDIR=/tmp):",
                     "", "    " + commands[f"trace_{w}"], "",
                     "| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
            for r in st[:14]:
                lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                             f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                             f"{float(r['Percentage']):.1f} % |")
            open(os.path.join(out_dir, f"kernels_{w}_trace.md"), "w").write("\n".join(lines) + "\n")
            printed += lines + [""]
        fe, wr = pmc(f"fetch_{w}", "FETCH_SIZE"), pmc(f"write_{w}", "WRITE_SIZE")
        if not (fe and wr and fetch_factor and write_factor):
            continue
        d = {"workload": WORKLOAD_TEXT[w], "fetch_calibration_factor": fetch_factor,
             "write_calibration_factor": write_factor, "operator_source_sha256_16": kernel_source_hash(),
             "commands": {k: v for k, v in commands.items() if k.endswith(w) or k.endswith("copy")}}
        txt = [f"# HBM traffic of the operator kernels, {WORKLOAD_TEXT[w]}", ""]
        for kind, fn in (("apply", apply_bytes), ("traction", traction_bytes)):
            kname = f"k_{kind}<{spec['p'] + 1}, double>"
            keys = [k for k in fe if kname in k]
            if not keys:
                continue
            f, wv = fe[keys[0]], wr[keys[0]]
            fb = float(np.mean(f)) * 1024.0 * fetch_factor
            wb = float(np.mean(wv)) * 1024.0 * write_factor
            d[kind] = {"kernel": kname.replace(" ", ""), "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                       "hbm_bytes_per_launch": fb + wb, "algorithmic_bytes_per_launch": fn(spec, 8)}
            txt += [f"`{kname.replace(' ', '')}`:", "",
                    f"FETCH_SIZE per launch {np.mean(f):.0f} KiB x {fetch_factor:.3f} = {fb / 1e6:.2f} MB",
                    f"WRITE_SIZE per launch {np.mean(wv):.0f} KiB x {write_factor:.3f} = {wb / 1e6:.2f} MB",
                    f"algorithmic bytes per launch {fn(spec, 8) / 1e6:.2f} MB "
                    f"(measured / algorithmic = {(fb + wb) / fn(spec, 8):.3f})", ""]
        txt += ["Calibration: the same counters on a plain copy of 256 MiB (bench.py --calib-copy) read "
                f"{max(cf):.0f} KiB fetched and {max(cw):.0f} KiB written per copy.", "", "Commands:", ""]
        txt += ["    " + c for c in d["commands"].values()]
        json.dump(d, open(os.path.join(out_dir, f"k_apply_{w}_traffic.json"), "w"), indent=1)
        open(os.path.join(out_dir, f"k_apply_{w}_traffic.md"), "w").write("\n".join(txt) + "\n")
        printed += txt + [""]
    s1, s4 = rows("solve_1", "run_kernel_stats.csv"), rows("solve_4", "run_kernel_stats.csv")
    if s1 and s4:
        a = {r["Name"]: r for r in s1}
        diff = []
        for r in s4:
            c1 = int(a[r["Name"]]["Calls"]) if r["Name"] in a else 0
            t1 = float(a[r["Name"]]["TotalDurationNs"]) if r["Name"] in a else 0.0
            dc, dt = int(r["Calls"]) - c1, float(r["TotalDurationNs"]) - t1
            if dc > 0:
                diff.append((dt, dc, r["Name"]))
        diff.sort(reverse=True)
        tot = sum(d[0] for d in diff)
        lines = [f"# Kernels of the solve loop alone, {WORKLOAD_TEXT[HEADLINE]}", "",
                 "Three passes of: FP32-preconditioned flexible CG to rtol 5e-8, layer energies, adjoint solve",
                 "and the forty coating-thickness derivatives. Setup (hierarchy, smoother data, coarsest",
                 "inverse) and the first pass (graph recording) are excluded: the figures are the",
                 "difference of a four-pass run and a one-pass run.", "",
                 "Commands (from the repository root, TMPDIR=/tmp):", "", "    " + commands["solve_4"],
                 "    " + commands["solve_1"], "",
                 f"Kernel time of the three passes: {tot / 1e6:.2f} ms", "",
                 "| kernel | calls | average (us) | total (ms) | share |", "|---|---|---|---|---|"]
        for dt, dc, name in diff[:24]:
            lines.append(f"| `{_short(name)}` | {dc} | {dt / dc / 1e3:.2f} | {dt / 1e6:.3f} | {100 * dt / tot:.1f} % |")
        open(os.path.join(out_dir, f"solve_loop_{HEADLINE}_trace.md"), "w").write("\n".join(lines) + "\n")
        printed += lines
    print("\n".join(printed))


def kernel_source_hash():
    """Hash of the sources the operator kernels are compiled from (kernels,
    device helpers, level view)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "element.h", "internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2111_06893_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(name, kind="apply"):
    """HBM bytes per launch of the FP64 operator kernel `kind` ("apply" or
    "traction") on workload `name` from the committed counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"k_apply_{name}_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("operator_source_sha256_16") != kernel_source_hash():
        return None
    return (d.get(kind) or {}).get("hbm_bytes_per_launch")


if __name__ == "__main__":
    main()
