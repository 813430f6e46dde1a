#!/usr/bin/env python3
"""Benchmark of the EFIE fill on one MI355X.

One step = one pass of the whole forward path in table mode on the 30,720-
unknown icosphere (20,480 triangles, k = 17 rad/m, 7-point rule, complex64
Z): exact FP64 distance range, FP64 table construction, geometry, FP64
touching pairs, FP32 regular-pair tile fill.  The direct-exponential fill of
the same matrix is timed beside it.  Prints one JSON line.
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

METRIC = "Z entries/s + Green evals/s, table vs direct-exp, at rel err ≤1e-5 vs FP64"
FLOPS_PER_EVAL = 40           # algorithmic FP32 flops per Green evaluation
PEAK_FP32 = 157.3             # TFLOP/s, MI355X FP32 vector peak
FILL_KERNEL_SRC = os.path.join(ROOT, "paper_1901_04162_amd", "csrc", "fill.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fill_table_ico5_traffic.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _traffic():
    """HBM bytes per fill launch from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    src = hashlib.sha256(open(FILL_KERNEL_SRC, "rb").read()).hexdigest()[:16]
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("fill_source_sha256_16") != src:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(V, F, edges, k, Q, seconds):
    """The oracle, untuned, on a sample of entries of the same matrix."""
    import numpy as np

    import oracle
    from paper_1901_04162_amd import meshes

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = 2000
    rows, cols = meshes.entry_sample(edges.shape[0], n, 101)
    t0 = time.perf_counter()
    oracle.fill_entries(V, F, edges, k, Q, rows, cols)
    dt = time.perf_counter() - t0
    n2 = int(min(5_000_000, max(n, n * seconds / max(dt, 1e-6))))
    rows, cols = meshes.entry_sample(edges.shape[0], n2, 102)
    t0 = time.perf_counter()
    oracle.fill_entries(V, F, edges, k, Q, rows, cols)
    dt = time.perf_counter() - t0
    return {
        "value": n2 / dt,
        "unit": "Z entries/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{n2} entries drawn uniformly from the same {edges.shape[0]}^2 matrix, "
                  f"FP64 direct exp, one entry at a time ({dt:.1f} s)",
        "green_evals_per_s": n2 * 4 * Q * Q / dt,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--subdiv", type=int, default=5)
    ap.add_argument("--k", type=float, default=17.0)
    ap.add_argument("--q", type=int, default=7)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the fill shards by row blocks across GPUs, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1901_04162_amd as mf
    from paper_1901_04162_amd import meshes

    torch.cuda.set_device(0)
    V, F = meshes.icosphere(args.subdiv)
    k, Q = args.k, args.q
    mesh = mf.Mesh(F, V.shape[0])
    E = mesh.n_edges
    T_ = F.shape[0]
    n_touch = mesh.n_touching()
    evals = (T_ * T_ - n_touch) * Q * Q  # regular quadrature-point pairs
    Vd = torch.tensor(V, dtype=torch.float64, device="cuda")
    Z = torch.empty((E, E), dtype=torch.complex64, device="cuda")
    log(f"workload: icosphere s={args.subdiv} T={T_} E={E} k={k} Q={Q} tol={args.tol}; "
        f"{evals:.4e} Green evals per fill")

    tabs = {}

    def step_table():
        lo, hi = mf.r_range(mesh, Vd, Q)
        tabs["T"] = mf.build_tables(k, lo, hi, args.tol)
        mf.fill_Z(mesh, Vd, k, Q, "table", tabs["T"], out=Z)

    def step_direct():
        mf.fill_Z(mesh, Vd, k, Q, "direct", out=Z)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        mf.set_timing(True)
        fill_ms = []
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
            fill_ms.append(mf.timings(mesh))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        mf.set_timing(False)
        mf.sync_status(mesh)
        return wall / steps, np.array(fill_ms)

    s_table, ph_table = timed(step_table, args.steps, args.warmup)
    log(f"table step {s_table*1e3:.2f} ms; phases (geom, touching, fill) ms "
        f"{ph_table.mean(0).round(3).tolist()}")
    T = tabs["T"]
    out = {
        "metric": METRIC,
        "value": E * E / s_table,
        "unit": "Z entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": s_table * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"icosphere r=1 m, {args.subdiv} subdivisions ({T_} triangles, {E} RWG "
                        f"unknowns), k={k} rad/m, {Q}-point rule, complex64 Z, table mode tol "
                        f"{args.tol}; step = distance range + tables + fill",
            "triangles": T_, "unknowns": E, "k": k, "quad_order": Q, "tol": args.tol,
            "green_table_samples": T.n_green, "green_table_buckets": T.m_green,
            "exp_table_samples": T.n_exp,
        },
        "green_evals_per_s": evals / s_table,
        "table_fill_only": {
            "ms": float(ph_table[:, 2].mean()),
            "z_entries_per_s": E * E / (ph_table[:, 2].mean() * 1e-3),
            "green_evals_per_s": evals / (ph_table[:, 2].mean() * 1e-3),
        },
        "phases_ms": {"geometry": float(ph_table[:, 0].mean()),
                      "touching_pairs_fp64": float(ph_table[:, 1].mean()),
                      "regular_fill": float(ph_table[:, 2].mean()),
                      "range_and_tables": float(s_table * 1e3 - ph_table.sum(1).mean())},
    }
    if not args.no_direct:
        s_direct, ph_direct = timed(step_direct, args.steps, args.warmup)
        log(f"direct step {s_direct*1e3:.2f} ms; phases {ph_direct.mean(0).round(3).tolist()}")
        out["direct"] = {
            "ms_per_step": s_direct * 1e3,
            "z_entries_per_s": E * E / s_direct,
            "green_evals_per_s": evals / s_direct,
            "regular_fill_ms": float(ph_direct[:, 2].mean()),
        }
        out["table_over_direct"] = s_direct / s_table
        out["table_over_direct_fill_only"] = float(ph_direct[:, 2].mean() / ph_table[:, 2].mean())
    fill_s = float(ph_table[:, 2].mean()) * 1e-3
    achieved = FLOPS_PER_EVAL * evals / fill_s / 1e12
    traffic = _traffic()
    out["roofline"] = {
        "bound": "alu",
        "kernel": "k_fill (table mode)",
        "achieved": achieved,
        "peak": PEAK_FP32,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32,
        "traffic": traffic,
        "flops_per_launch": FLOPS_PER_EVAL * evals,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(V, F, mesh.edges(), k, Q, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
