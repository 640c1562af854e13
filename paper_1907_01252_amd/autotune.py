"""Autotuner of the fine propagator's launch and schedule choices.

    python -m paper_1907_01252_amd.autotune c2:32 c3:8 c5:4 [--reps 2]

(workload[:steps per slice], default --steps-per-slice)

On the GPU it is run on, for each named workload (synth.workload), the tuner
times a short fine sweep of the workload's full size (all slices in one
fine_propagate call, `steps_per_slice` steps of the workload's step size, the
inputs from a one-step coarse sweep) under candidate settings of the choices
that change how the work is launched but not what is computed:

  batch_split       concurrent slice groups (1, 2 or 3; also 4 when the process
                    has at least 8 hardware queues, GPU_MAX_HW_QUEUES: each group's
                    stream needs one of its own, and HIP's default is 4)
  spmv_slice_fast   SpMV grid with the slices as the fast dimension (0 or 1)
  vanka_slice_fast  the same for the fused Vanka pass (0 or 1)
  vanka_wide_cells  3d only: colour size over the batch from which the fused
                    Vanka pass takes 32 cells per block instead of 8

It searches them one at a time (coordinate descent from the built-in defaults,
each candidate timed as the best of `reps` sweeps after a warm-up sweep on a
fresh problem), and keeps a candidate only if it is faster by more than 1%.
Every candidate's output is compared with the first configuration's; the
largest relative difference is recorded (the choices reorder launches, so it
is zero unless a choice changes the arithmetic).

The result goes to tuned.json next to this file, keyed by the problem's
dimension, refinement level, precision and batch size and by the process's
hardware queue count (no suffix for HIP's default of 4, -q<N> otherwise), which
make_params() applies to a problem of that key unless the caller sets a choice
itself; the timings of every candidate go to profiles/autotune_<workload>.md
(autotune_<workload>_q<N>.md).
"""
from __future__ import annotations

import argparse
import datetime
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TABLE = os.path.join(HERE, "tuned.json")

CHOICES = ("batch_split", "spmv_slice_fast", "vanka_slice_fast", "vanka_wide_cells")


def hw_queues() -> int:
    """Hardware queues HIP gives this process (GPU_MAX_HW_QUEUES, default 4)."""
    try:
        return max(1, int(os.environ.get("GPU_MAX_HW_QUEUES", "4")))
    except ValueError:
        return 4


def candidates(dim: int, queues: int = 4) -> dict:
    # five or more groups measured about twice as slow as four, with 8 or 16 queues
    c = {"batch_split": [1, 2, 3] + ([4] if queues >= 8 else []), "spmv_slice_fast": [0, 1],
         "vanka_slice_fast": [0, 1]}
    if dim == 3:
        c["vanka_wide_cells"] = [4096, 8192, 16384, 1 << 30]
    return c


def table_key(dim: int, level: int, precision: str, max_batch: int, queues: int = 4) -> str:
    return f"d{dim}-l{level}-{precision}-b{max_batch}" + ("" if queues == 4 else f"-q{queues}")


def load_table() -> dict:
    if not os.path.exists(TABLE):
        return {}
    with open(TABLE) as f:
        return json.load(f)


def builtin_defaults(dim: int, precision: str) -> dict:
    """The library's own choices for the -1 / 0 settings (for the starting point)."""
    fp64 = precision == "fp64"
    return {"batch_split": 3, "spmv_slice_fast": 1 if (dim == 2 and fp64) else 0,
            "vanka_slice_fast": 1 if (dim == 3 or fp64) else 0, "vanka_wide_cells": 8192}


class _Sweep:
    """Inputs and a timed fine sweep of one workload (GPU)."""

    def __init__(self, name: str, steps_per_slice: int):
        import torch
        import synth
        from . import fsi
        self.torch, self.fsi = torch, fsi
        self.p = p = synth.workload(name, seed=0)
        self.name = name
        self.prec = p["precision"]
        self.N, self.m = p["N"], steps_per_slice
        self.dl = p["slice_len"] * steps_per_slice / p["m"]
        prob = fsi.Problem(fsi.make_params(p, max_batch=self.N, tuned=False))
        nc = prob.n_dofs // prob.n_nodes
        U = torch.zeros(self.N + 1, prob.n_nodes, nc, dtype=torch.float64, device="cuda")
        prob.initial_state(U[0])
        for l in range(self.N):
            out = torch.zeros_like(U[0:1])
            prob.coarse_propagate(1, [l * self.dl], self.dl, 1, U[l:l + 1].contiguous(), out)
            U[l + 1] = out[0]
        prob.close()
        self.Uin = U[:self.N].contiguous()
        self.t0s = [l * self.dl for l in range(self.N)]
        self.ref = None

    def time(self, choice: dict, reps: int):
        torch, fsi = self.torch, self.fsi
        prob = fsi.Problem(fsi.make_params(self.p, max_batch=self.N, tuned=False, **choice))
        out = torch.zeros_like(self.Uin)
        prob.fine_propagate(self.N, self.t0s, self.dl, self.m, self.Uin, out)   # warm-up (workspaces, graphs)
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, st = prob.fine_propagate(self.N, self.t0s, self.dl, self.m, self.Uin, out)
            torch.cuda.synchronize()
            w = time.perf_counter() - t
            best = w if best is None else min(best, w)
        prob.close()
        res = out.cpu().numpy()
        if self.ref is None:
            self.ref = res
        diff = float(np.abs(res - self.ref).max() / max(np.abs(self.ref).max(), 1e-300))
        return best, diff, (st.newton_total, st.krylov_total)


def tune(name: str, steps_per_slice: int = 4, reps: int = 2, log=print) -> dict:
    sw = _Sweep(name, steps_per_slice)
    dim = sw.p["dim"]
    cur = builtin_defaults(dim, sw.prec)
    if dim != 3:
        cur.pop("vanka_wide_cells")
    trials = []
    best_t, diff, counts = sw.time(cur, reps)
    trials.append({"choice": dict(cur), "seconds": best_t, "max_rel_diff": diff, "newton_krylov": counts})
    q = hw_queues()
    log(f"autotune {name}: start {cur} {best_t:.4f} s ({q} hardware queues)")
    for key, values in candidates(dim, q).items():
        for v in values:
            if v == cur[key]:
                continue
            trial = dict(cur)
            trial[key] = v
            t, diff, counts = sw.time(trial, reps)
            trials.append({"choice": trial, "seconds": t, "max_rel_diff": diff, "newton_krylov": counts})
            log(f"autotune {name}: {key}={v} {t:.4f} s (best {best_t:.4f}), max rel diff {diff:.1e}")
            if t < 0.99 * best_t:
                cur, best_t = trial, t
    p = sw.p
    return {"workload": name, "key": table_key(dim, p["level"], sw.prec, sw.N, q), "queues": q,
            "choice": cur, "seconds": best_t,
            "sweep": f"{name}: {sw.N} slices x {steps_per_slice} steps of {p['k_fine']:.6g}, {sw.prec}",
            "reps": reps, "trials": trials,
            "date": datetime.datetime.now(datetime.timezone.utc).strftime("%Y-%m-%d %H:%M UTC")}


def _evidence(r: dict) -> str:
    return f"autotune_{r['workload']}" + ("" if r["queues"] == 4 else f"_q{r['queues']}") + ".md"


def write(results: list, table_path: str = TABLE, profiles: str | None = None, command: str = ""):
    table = load_table() if table_path == TABLE else {}
    for r in results:
        table[r["key"]] = {"workload": r["workload"], "choice": r["choice"], "seconds": r["seconds"],
                           "sweep": r["sweep"], "hw_queues": r["queues"], "evidence": f"profiles/{_evidence(r)}"}
    with open(table_path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    if profiles:
        for r in results:
            lines = [f"# Autotuner: {r['sweep']}, {r['queues']} hardware queues", "",
                     "Command (repository root, one MI355X):", "", f"    {command}", "",
                     f"Measured {r['date']}; each row is the best of {r['reps']} sweeps after a warm-up sweep on a "
                     "fresh problem. Coordinate descent from the built-in defaults (first row); a candidate is kept "
                     "when it is more than 1% faster. The last column is the largest relative difference of the "
                     "sweep's output from the first row's.", "",
                     f"Chosen: `{json.dumps(r['choice'])}` ({r['seconds'] * 1e3:.1f} ms per sweep), stored under "
                     f"`{r['key']}` in `paper_1907_01252_amd/tuned.json`.", "",
                     "| choice | ms per sweep | Newton, Krylov | max rel. diff |", "|---|---|---|---|"]
            for t in r["trials"]:
                lines.append(f"| `{json.dumps(t['choice'])}` | {t['seconds'] * 1e3:.1f} | "
                             f"{t['newton_krylov'][0]}, {t['newton_krylov'][1]} | {t['max_rel_diff']:.1e} |")
            with open(os.path.join(profiles, _evidence(r)), "w") as f:
                f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="+")
    ap.add_argument("--steps-per-slice", type=int, default=4)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--out", default=TABLE, help="table to write (default: the package's tuned.json)")
    ap.add_argument("--profiles", default=os.path.join(ROOT, "profiles"),
                    help="directory of the evidence summaries ('' for none)")
    a = ap.parse_args()
    sys.path.insert(0, ROOT)
    # the command as run with the default outputs (this package's tuned.json, profiles/)
    q = hw_queues()
    cmd = (f"GPU_MAX_HW_QUEUES={q} " if q != 4 else "") + \
        f"python -m paper_1907_01252_amd.autotune {' '.join(a.workloads)} --reps {a.reps}"
    res = []
    for spec in a.workloads:
        name, _, steps = spec.partition(":")
        res.append(tune(name, int(steps) if steps else a.steps_per_slice, a.reps, log=lambda s: print(s, flush=True)))
        write(res, a.out, a.profiles or None, cmd)   # after every workload: partial results survive
    print(json.dumps({r["workload"]: r["choice"] for r in res}))


if __name__ == "__main__":
    main()
