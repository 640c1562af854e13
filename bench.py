"""Fine-propagator throughput on one MI355X.

Workload (default): 2d ALE-FSI channel with an elastic bar, 128x32 Q1 cells
(21,285 unknowns), 32 Parareal slices of length 1/16 on [0, 2], 32 shifted
Crank-Nicolson steps of 2^-9 per slice, FP64.  The slice inputs are the
states of the initial coarse sweep (4 coarse steps per slice), i.e. the inputs
of the first Parareal fine sweep.  One timed step = one batched fine sweep
(fine_propagate over all 32 slices).  Reported:

  value            dof.steps/s of the batched sweep (unknowns x steps x slices / wall time)
  sequential       slices spread over [0, T] propagated one call per slice
                   (B = 1), same solver settings; their outputs must equal the
                   timed batched sweep's outputs of the same slices (1e-10 per
                   field in FP64, 1e-6 mixed)
  roofline         the colored Vanka smoothing pass (dominant kernel): algorithmic
                   bytes per launch (active slices only) / mean launch time from
                   HIP events on the library's stream, against the 8 TB/s HBM peak
  roofline_c3/_c5  the same for the 256x64 mixed and the 64x16x16 3d workloads
                   (short sweeps, same kernels and sizes)
  accuracy         a batched-sweep slice against the FP64 oracle on a bounded
                   number of steps (gate 1e-10 relative per field in FP64, 1e-6 mixed)
  cpu_baseline     the oracle (NumPy/SciPy, SuperLU) on the host, same slice,
                   bounded to a few steps; slice_parallel: one process per slice
                   on up to 16 host cores, the same few steps each
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# Each concurrent slice group of a propagator call runs on a stream of its own, which needs a
# hardware queue of its own; HIP gives a process 4 by default, and the benchmark asks for at
# least 8 before the HIP runtime starts (the autotuned choices are stored per queue count).
try:
    _hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
except ValueError:
    _hwq = 4
os.environ["GPU_MAX_HW_QUEUES"] = str(max(_hwq, 8))

HBM_PEAK_GBS = 8000.0
METRIC = "fine-propagator dof\u00b7steps/s batched vs sequential slices at 1e-6 rel; HBM GB/s"
# kernel families timed by the library (HIP events on the call's stream), in fsi_profile_query order
FAMILIES = ("vanka_pass_fine", "krylov_spmv_fine", "jacobian_elem", "residual", "level_residual_fine",
            "coarser_levels", "coarsest_solve")
KERNEL_NAMES = {"vanka_pass_fine": "k_vanka_color (fused residual + patch update, finest level)",
                "krylov_spmv_fine": "k_spmv (Krylov product, finest level)",
                "level_residual_fine": "k_spmv (residual before restriction, finest level)"}


def counter_traffic(workload, kernel_family, prec):
    """HBM bytes per launch of the dominant kernel from the committed counter runs, or None.

    profiles/traffic.json records, per workload, the FETCH_SIZE/WRITE_SIZE means of
    the kernel's launches over the whole batch (calibrated with a copy kernel), and a
    hash of the kernel's source at the time of the runs; another family, precision or
    a changed kernel gives None.
    """
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    w = tr.get("workloads", {}).get(workload)
    if w is None or tr.get("family") != kernel_family or w.get("precision") != prec:
        return None
    if kernel_source_hash(tr["kernel_function"]) != tr["source_hash"]:
        return None
    return w["traffic_bytes_per_launch"]


def kernel_source_hash(fn):
    """Hash of the dominant kernel's source (vanka.hip, which holds the kernel, stencil.h
    with its device helpers, and the shared layout header with the storage of the
    Jacobian and of the inverses it reads), tagged with the kernel name: any edit there
    invalidates counter figures taken before it."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1907_01252_amd", "csrc")
    src = "".join(open(os.path.join(csrc, f)).read() for f in ("vanka.hip", "stencil.h", "fsi_internal.h"))
    assert f" {fn}(" in src, fn
    return hashlib.sha256((fn + src).encode()).hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default=None, help="fp64 | mixed (default: the workload's)")
    ap.add_argument("--seq-slices", type=int, default=4,
                    help="slices of the sequential baseline, spread evenly over the interval")
    ap.add_argument("--gate-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-seq", action="store_true")
    ap.add_argument("--steps-per-slice", type=int, default=None,
                    help="override m (shorter sweeps for hardware-counter runs; same kernels and sizes)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before the sweep, copy this many MB with a plain device copy (counter calibration)")
    ap.add_argument("--no-profile-sweep", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the short profiled c3 and c5 sweeps (roofline_c3, roofline_c5)")
    ap.add_argument("--progress", action="store_true",
                    help="print a line to stderr after each fine sweep (long profiler runs)")
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="most host processes of the slice-parallel oracle figure")
    ap.add_argument("--set", action="append", default=[], metavar="KEY=VALUE",
                    help="solver parameter override (fsi_params field), e.g. vanka_sweeps_coarse=1")
    ap.add_argument("--parareal", action="store_true",
                    help="time parareal_run on the c1 workload, plain and pipelined schedules")
    ap.add_argument("--adjoint", action="store_true",
                    help="time one adjoint_gradient call of the c4 workload instead of the fine sweep")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the fine propagator runs on one GPU: the sweep's slices are batched on a single "
                                   "MI355X; multi-GPU runs are not part of it", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import synth
    from paper_1907_01252_amd import fsi

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.adjoint:
        return adjoint_bench(args)
    if args.parareal:
        return parareal_bench(args)
    p = synth.workload(args.workload, seed=0)
    prec = args.precision or p["precision"]
    N, m, M, dl = p["N"], p["m"], p["M"], p["slice_len"]
    if args.steps_per_slice:
        dl = dl * args.steps_per_slice / m
        m, M = args.steps_per_slice, 1
    overrides = {kv.split("=")[0]: float(kv.split("=")[1]) for kv in args.set}
    prob = fsi.Problem(fsi.make_params(p, precision=prec, max_batch=N, **overrides))
    nd = prob.n_dofs
    dev = "cuda"

    # ---- inputs: initial coarse sweep (untimed setup)
    nc = prob.n_dofs // prob.n_nodes
    dim = p["dim"]
    U = torch.zeros(N + 1, prob.n_nodes, nc, dtype=torch.float64, device=dev)
    prob.initial_state(U[0])
    for l in range(N):
        out = torch.zeros_like(U[0:1])
        prob.coarse_propagate(1, [l * dl], dl, M, U[l:l + 1].contiguous(), out)
        U[l + 1] = out[0]
    Uin = U[:N].contiguous()
    t0s = [l * dl for l in range(N)]
    Uout = torch.zeros_like(Uin)

    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- warmup + timed batched sweeps
    def say(msg):
        if args.progress:
            print(f"bench: {msg}", file=sys.stderr, flush=True)

    say(f"inputs ready ({args.workload}, {N} slices x {m} steps)")
    for w in range(args.warmup):
        prob.fine_propagate(N, t0s, dl, m, Uin, Uout)
        say(f"warm-up sweep {w + 1} done")
    torch.cuda.synchronize()
    t_a = time.perf_counter()
    stats = []
    for q in range(args.steps):
        _, st = prob.fine_propagate(N, t0s, dl, m, Uin, Uout)
        stats.append((st.newton_total, st.krylov_total))
        say(f"timed sweep {q + 1} done")
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    wall = (t_b - t_a) / args.steps
    Ubatch = Uout.clone()
    # one more sweep of the same workload with HIP events around every launch of the
    # profiled kernel families (kernels launched directly, not replayed from graphs; the
    # library runs it as one batch of all slices, so that no other group's kernels share
    # the GPU with a timed launch)
    prof_wall = 0.0
    fams = {name: (0, 0.0, 0.0) for name in FAMILIES}
    if not args.no_profile_sweep:
        prob.profile_enable(True)
        t_p = time.perf_counter()
        prob.fine_propagate(N, t0s, dl, m, Uin, Uout)
        torch.cuda.synchronize()
        prof_wall = time.perf_counter() - t_p
        prob.profile_enable(False)
        fams = {name: prob.profile_query(i) for i, name in enumerate(FAMILIES)}
    dof_steps = nd * m * N
    value = dof_steps / wall

    # ---- sequential-slice path (B = 1 calls) on slices spread over the whole interval; its
    # outputs must equal the timed batched sweep's outputs of the same slices
    seq = None
    eq_tol = 1e-10 if prec == "fp64" else 1e-6
    if not args.no_seq:
        S = min(args.seq_slices, N)
        picks = sorted({int(round(q * (N - 1) / max(S - 1, 1))) for q in range(S)})
        outs = {}
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        for l in picks:
            o = torch.zeros_like(Uin[l:l + 1])
            prob.fine_propagate(1, [t0s[l]], dl, m, Uin[l:l + 1].contiguous(), o)
            outs[l] = o
        torch.cuda.synchronize()
        seq_wall = time.perf_counter() - t_c
        diff = 0.0
        for l in picks:
            a, b = outs[l][0].cpu().numpy(), Ubatch[l].cpu().numpy()
            for sl in fields(dim).values():
                diff = max(diff, float(np.linalg.norm(a[:, sl] - b[:, sl]) / max(np.linalg.norm(b[:, sl]), 1e-300)))
        seq = {"value": nd * m * len(picks) / seq_wall, "slices_timed": picks, "ms_per_slice": 1e3 * seq_wall / len(picks),
               "max_rel_diff_vs_batched": diff, "gate": eq_tol, "pass": diff <= eq_tol}

    # ---- accuracy gate and CPU baseline: oracle on slice 1 for a few steps
    acc, cpu = None, None
    # the 3d oracle needs minutes per Newton step at the benchmark size: no CPU leg there
    if not args.no_cpu and dim == 2:
        from oracle.residual import Discretization
        from oracle import propagate as P
        D = Discretization(p)
        k = p["k_fine"]
        l = 1
        u_in = Uin[l].cpu().numpy()
        ns = args.gate_steps
        threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
        # the oracle first, bounded by --cpu-seconds (at least one step); the GPU then takes
        # exactly the steps the oracle finished, so the gate is reported at any workload size
        t_d = time.perf_counter()
        c_d = time.process_time()
        ref = u_in
        done = 0
        for n in range(ns):
            ref = P.newton_step(D, ref, t0s[l] + (n + 1) * k, k)
            done += 1
            if time.perf_counter() - t_d > args.cpu_seconds:
                break
        cpu_wall = time.perf_counter() - t_d
        # cores actually busy: process CPU time (all threads) over wall time
        cores_used = max(1, int(round((time.process_time() - c_d) / cpu_wall)))
        # GPU: the same slice, same input, the same steps (B = 1 call of the product path)
        o = torch.zeros_like(Uin[l:l + 1])
        prob.fine_propagate(1, [t0s[l]], done * k, done, Uin[l:l + 1].contiguous(), o)
        g = o[0].cpu().numpy()
        errs = {}
        for f, sl in fields(dim).items():
            errs[f] = float(np.linalg.norm(g[:, sl] - ref[:, sl]) / np.linalg.norm(ref[:, sl]))
        acc = {"max_rel_err": max(errs.values()), "per_field": errs, "gate": eq_tol,
               "pass": max(errs.values()) <= eq_tol, "sample": f"slice {l}, {done} steps vs FP64 oracle"}
        cpu = {"value": nd * done / cpu_wall, "unit": "dof\u00b7steps/s", "cores": cores_used,
               "threads_allowed": int(threads), "kind": "oracle",
               "sample": f"slice {l} of {args.workload}: {done} Newton-SuperLU steps, {cpu_wall:.1f} s"}
        # the same number of steps per process as the single-process figure finished (bounded likewise)
        cpu["slice_parallel"] = oracle_slice_parallel(args.workload, [Uin[q].cpu().numpy() for q in range(N)], t0s, k,
                                                      done, args.cpu_procs, nd)

    roof = roofline_of(fams, lambda fam, pr: counter_traffic(args.workload, fam, pr), prec)
    ej = element_jacobian_roof(prob, p, N) if not args.no_extra else None
    prob.close()
    extra = {}
    if not args.no_extra and args.workload == "c2":
        for name, msteps in (("c3", 4), ("c5", 2)):
            extra["roofline_" + name] = short_profiled_roofline(name, msteps)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "dof\u00b7steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32-inner/f64-newton",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {dim}d ALE-FSI {'channel+bar' if dim == 2 else 'duct+block'}, "
                               f"{p['level']}-level-refined {'x'.join(str(c) for c in synth.mesh_shape(p))} "
                               f"Q{p.get('degree', 1)}, "
                               f"{nd} unknowns, {N} slices x {m} steps of {p['k_fine']:.6g}",
                   "slices": N, "steps_per_slice": m, "unknowns": nd, "precision": prec,
                   "batch_split": int(prob.params.batch_split),
                   "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"]),
                   "launch": {k: int(getattr(prob.params, k)) for k in ("spmv_slice_fast", "vanka_slice_fast",
                                                                         "vanka_wide_cells")},
                   "solver_overrides": overrides},
        "newton_per_sweep": stats[-1][0], "krylov_per_sweep": stats[-1][1],
        "sequential": seq,
        "speedup_batched_vs_sequential": (value / seq["value"]) if seq else None,
        "roofline": roof,
        "element_jacobian": ej,
        **extra,
        "profiled_sweep_ms": 1e3 * prof_wall,
        "kernels": {f: {"launches": v[0], "ms_per_sweep": v[1],
                        "GBs": (v[2] / (v[1] * 1e-3) / 1e9) if v[1] > 0 else None} for f, v in fams.items()},
        "accuracy": acc,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def fields(dim):
    return {"v": slice(0, dim), "u": slice(dim, 2 * dim), "p": slice(2 * dim, 2 * dim + 1)}


def roofline_of(fams, traffic_fn, prec):
    """roofline object of the dominant kernel family (largest time in the profiled sweep)."""
    dom = max(("vanka_pass_fine", "krylov_spmv_fine", "level_residual_fine"), key=lambda f: fams[f][1])
    dn, dms, dby = fams[dom]
    achieved = dby / (dms * 1e-3) / 1e9 if dms > 0 else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": traffic_fn(dom, prec) if traffic_fn else None,
            "kernel": KERNEL_NAMES.get(dom, dom), "launches": dn,
            "mean_launch_us": 1e3 * dms / max(dn, 1), "bytes_per_launch": dby / max(dn, 1),
            "measured_on": "profiled sweep: all slices in one batch, HIP events around every launch; "
                           "bytes of the slices each launch works on"}


FP64_VECTOR_PEAK_TFS = 78.6


def element_jacobian_roof(prob, p, B):
    """The element Jacobian (k_elem_jacobian) against both roofs: the element matrices of every
    level for B slices, assembled by fsi_debug_jacobian_apply at random admissible states under HIP
    events (profiled family jacobian_elem).  FP64 operations per cell: the committed FP64
    instruction counts of the kernel (profiles/flops.json, 64 lanes per wave instruction, an FMA
    two operations); bytes: the element matrices written and the two states read.  Q1 only."""
    import torch
    import synth
    if p.get("degree", 1) != 1:
        return None
    path = os.path.join(ROOT, "profiles", "flops.json")
    if not os.path.exists(path):
        return None
    dim = p["dim"]
    per_cell = json.load(open(path))["k_elem_jacobian"][f"{dim}d"]["flop_per_cell"]
    shape = synth.mesh_shape(p)
    ncell = int(np.prod(shape))
    cells = B * sum(ncell // (2 ** dim) ** j for j in range(p["level"] + 1))
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    U = dev(np.stack([synth.random_state(p, 900 + b, grad_u_max=0.02) for b in range(B)]))
    Uo = dev(np.stack([synth.random_state(p, 950 + b, grad_u_max=0.02) for b in range(B)]))
    X = dev(np.stack([synth.random_state(p, 990 + b) for b in range(B)]))
    Y = torch.zeros_like(X)
    t = [0.1] * B
    prob.debug_jacobian_apply(B, U, Uo, t, p["k_fine"], X, Y)     # warm-up
    best = None
    for _ in range(3):
        prob.profile_enable(True)
        prob.debug_jacobian_apply(B, U, Uo, t, p["k_fine"], X, Y)
        torch.cuda.synchronize()
        n, ms, by = prob.profile_query(FAMILIES.index("jacobian_elem"))
        prob.profile_enable(False)
        if best is None or ms < best[1]:
            best = (n, ms, by)
    n, ms, by = best
    tfs = per_cell * cells / (ms * 1e-3) / 1e12
    gbs = by / (ms * 1e-3) / 1e9
    return {"bound": "alu", "achieved": tfs, "peak": FP64_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
            "frac": tfs / FP64_VECTOR_PEAK_TFS, "hbm_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "kernel": f"k_elem_jacobian<{dim}, false>", "launches": n, "ms_all_levels": ms, "cells": cells,
            "flop_per_cell": per_cell,
            "measured_on": f"element matrices of all {p['level'] + 1} levels, {B} slices, HIP events; "
                           "FP64 operations per cell from counted instructions"}


def short_profiled_roofline(name, msteps):
    """Dominant-kernel roofline of a short profiled sweep of workload `name` (msteps fine steps of
    the workload's size per slice, all slices in one batch; inputs from a one-step coarse sweep)."""
    import torch
    import synth
    from paper_1907_01252_amd import fsi
    p = synth.workload(name, seed=0)
    prec = p["precision"]
    N, m = p["N"], p["m"]
    dl = p["slice_len"] * msteps / m
    prob = fsi.Problem(fsi.make_params(p, precision=prec, max_batch=N))
    nc = prob.n_dofs // prob.n_nodes
    U = torch.zeros(N + 1, prob.n_nodes, nc, dtype=torch.float64, device="cuda")
    prob.initial_state(U[0])
    for l in range(N):
        out = torch.zeros_like(U[0:1])
        prob.coarse_propagate(1, [l * dl], dl, 1, U[l:l + 1].contiguous(), out)
        U[l + 1] = out[0]
    Uin = U[:N].contiguous()
    Uout = torch.zeros_like(Uin)
    t0s = [l * dl for l in range(N)]
    prob.fine_propagate(N, t0s, dl, msteps, Uin, Uout)      # warm-up
    prob.profile_enable(True)
    _, st = prob.fine_propagate(N, t0s, dl, msteps, Uin, Uout)
    torch.cuda.synchronize()
    prob.profile_enable(False)
    fams = {f: prob.profile_query(i) for i, f in enumerate(FAMILIES)}
    ej = element_jacobian_roof(prob, p, N)
    prob.close()
    r = roofline_of(fams, lambda fam, pr: counter_traffic(name, fam, pr), prec)
    r["element_jacobian"] = ej
    r["sweep"] = f"{name}: {prob.n_dofs} unknowns, {N} slices x {msteps} steps of {p['k_fine']:.6g}, {prec}"
    r["newton"], r["krylov"] = st.newton_total, st.krylov_total
    return r


def _oracle_slice_worker(name, u_in, t0, k, ns, barrier, queue):
    """One host process of the slice-parallel oracle figure: ns Newton-SuperLU steps of one slice."""
    from threadpoolctl import threadpool_limits
    import synth
    from oracle.residual import Discretization
    from oracle import propagate as P
    with threadpool_limits(1):
        D = Discretization(synth.workload(name, seed=0))
        barrier.wait()
        t_0 = time.perf_counter()
        U = u_in
        for n in range(ns):
            U = P.newton_step(D, U, t0 + (n + 1) * k, k)
        queue.put(time.perf_counter() - t_0)


def oracle_slice_parallel(name, inputs, t0s, k, ns, max_procs, nd):
    """The paper's one-slice-per-core model with the oracle: P processes (P = min(slices, host
    cores, max_procs)) each take ns steps of its own slice at the same time; throughput = P ns
    unknowns-steps over the slowest process's time.  A sample of the sweep (ns of m steps)."""
    import multiprocessing as mp
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    P = max(1, min(len(inputs), cores, max_procs))
    ctx = mp.get_context("spawn")
    barrier, queue = ctx.Barrier(P), ctx.Queue()
    picks = [int(round(q * (len(inputs) - 1) / max(P - 1, 1))) for q in range(P)]
    procs = [ctx.Process(target=_oracle_slice_worker, args=(name, inputs[l], t0s[l], k, ns, barrier, queue))
             for l in picks]
    for pr in procs:
        pr.start()
    walls = [queue.get(timeout=600) for _ in procs]
    for pr in procs:
        pr.join()
    return {"value": P * ns * nd / max(walls), "unit": "dof\u00b7steps/s", "cores": P, "processes": P,
            "kind": "oracle",
            "sample": f"{P} slices of {name} at once, one process each, {ns} Newton-SuperLU steps per slice "
                      f"(slowest {max(walls):.1f} s)"}


def adjoint_bench(args):
    """One adjoint_gradient call: J = time-integrated drag over [0, T], gradient w.r.t. (peak, mu_s, lambda_s)."""
    import torch
    import synth
    from paper_1907_01252_amd import fsi
    name = "c4" if args.workload == "c2" else args.workload
    p = synth.workload(name, seed=0)
    prob = fsi.Problem(fsi.make_params(p, precision="fp64", max_batch=p["N"]))
    U0 = torch.zeros(prob.n_nodes, prob.n_dofs // prob.n_nodes, dtype=torch.float64, device="cuda")
    prob.initial_state(U0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, g, st = prob.adjoint_gradient(p["T"], p["N"], p["m"], U0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps = p["N"] * p["m"]
    print(json.dumps({
        "metric": "adjoint gradient of the time-integrated drag: wall time of one call",
        "value": wall, "unit": "s", "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{name}: 2d ALE-FSI, {prob.n_dofs} unknowns, {p['N']} slices x {p['m']} steps, T={p['T']}"},
        "J": J, "grad": {"inflow_peak": g[0], "mu_s": g[1], "lambda_s": g[2]},
        "newton_forward": st.newton_total, "krylov_total": st.krylov_total,
        "krylov_backward": st.krylov_its[0], "steps": steps, "ms_per_backward_step": None,
    }))


def parareal_bench(args):
    """parareal_run on c1 (8 slices, tolerance 1e-8): the plain schedule (batched fine sweep, then the
    sequential correction sweep) against the pipelined one (fine chunks of G slices on a second stream,
    overlapped with the correction sweep), same iterates."""
    import torch
    import synth
    from paper_1907_01252_amd import fsi
    name = "c1" if args.workload == "c2" else args.workload
    p = synth.workload(name, seed=0)
    N = p["N"]
    rows = {}
    ref = None
    for G in [0, 1, 2, 4]:
        prob = fsi.Problem(fsi.make_params(p, max_batch=N, parareal_pipeline=G))
        nd = prob.n_dofs // prob.n_nodes
        U0 = torch.zeros(prob.n_nodes, nd, dtype=torch.float64, device="cuda")
        prob.initial_state(U0)
        Ub = torch.zeros(N + 1, prob.n_nodes, nd, dtype=torch.float64, device="cuda")
        best = None
        for rep in range(1 + args.steps):   # the first call also builds the worker workspace
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            code, st = prob.parareal_run(p["T"], N, p["m"], p["M"], 1e-8, N, U0, Ub, raise_on_error=False)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if rep > 0:
                best = wall if best is None else min(best, wall)
        U = Ub.cpu()
        if ref is None:
            ref = U
        rows[f"G{G}" if G else "plain"] = {
            "seconds": best, "iterations": st.parareal_iters, "status": int(code),
            "coarse_ms": st.stage_ms[5], "fine_ms": st.stage_ms[6],
            "max_rel_diff_vs_plain": float((U - ref).abs().max() / ref.abs().max()),
        }
        prob.close()
    plain = rows["plain"]["seconds"]
    bestG = min((k for k in rows if k != "plain"), key=lambda k: rows[k]["seconds"])
    print(json.dumps({
        "metric": "parareal_run wall time to tolerance 1e-8, plain vs pipelined schedule",
        "value": rows[bestG]["seconds"], "unit": "s", "higher_is_better": False, "n_gpus": 1, "dtype": "f64",
        "data": "synthetic", "config": {"workload": f"{name}: 2d ALE-FSI, {N} slices x {p['m']} fine / {p['M']} "
                                                   f"coarse steps, T={p['T']}"},
        "speedup_vs_plain": plain / rows[bestG]["seconds"], "best": bestG, "schedules": rows,
    }))


if __name__ == "__main__":
    main()
