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
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Z entries/s + Green evals/s, table vs direct-exp, at rel err ≤1e-5 vs FP64"
# Algorithmic FP32 flops per regular quadrature-point pair in table mode (an FMA
# counts 2): distance 8, R from rsqrt 1, bucket 2, offset 1, complex cubic
# 12, four complex moment sums 16.
FLOPS_PER_EVAL = 40
PEAK_FP32 = 157.3             # TFLOP/s, MI355X FP32 vector peak
FILL_KERNEL_SRC = os.path.join(ROOT, "paper_1901_04162_amd", "csrc", "fill.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fill_tb_ico5_traffic.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _traffic():
    """HBM bytes per launch of the tile kernel and of the cut-edge fix-up from
    the committed counter summary, if it was taken on the current kernel
    source; else (None, None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, None
    src = hashlib.sha256(open(FILL_KERNEL_SRC, "rb").read()).hexdigest()[:16]
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("fill_source_sha256_16") != src:
        return None, None
    try:
        return float(vals["hbm_bytes_per_launch"]), float(vals["fixup_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None, None


def _lscpu():
    """Host CPU description (model, sockets, cores, threads) from lscpu."""
    import subprocess

    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    keep = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)",
            "CPU max MHz", "L3 cache")
    out = {}
    for line in txt.splitlines():
        if ":" in line:
            key, val = line.split(":", 1)
            if key.strip() in keep:
                out[key.strip()] = val.strip()
    return out


def cpu_baseline(V, F, edges, k, Q, tol, seconds, sample=None):
    """The oracle, untuned, timed on the host cores, and the parity of the
    timed GPU fills.

    Rate: rows of the same matrix filled in triangle-pair order (each pair's
    kernel values evaluated once for its nine local entries), FP64 direct
    exponential, on all cores; a contiguous row block sized from a short
    calibration to take about `seconds`/2.  The same block in table mode (the
    oracle's Lagrange table, tol as the GPU) gives the oracle's own
    table-versus-direct ratio, and a smaller block on one thread the rate to
    set beside the paper's single-threaded CPU.

    Parity: `sample` = (flat indices, {mode: GPU values}); the oracle's
    entries at those indices give the relative Frobenius error of each timed
    fill and the element-wise relative errors of the real and imaginary
    parts."""
    import numpy as np

    import oracle

    E = edges.shape[0]
    threads = oracle.max_threads()

    def rate(r0, r1, mode=oracle.DIRECT, G=None):
        t0 = time.perf_counter()
        oracle.fill_rows(V, F, edges, k, Q, r0, r1, mode=mode, gtable=G)
        return time.perf_counter() - t0

    dt = rate(0, 32)
    rows = int(min(E, max(32, 32 * 0.5 * seconds / max(dt, 1e-6))))
    dt = rate(0, rows)
    lo, hi = oracle.r_range(V, F, Q)
    G = oracle.build_table(oracle.GREEN, k, lo, hi, tol)
    dt_table = rate(0, rows, oracle.TABLE, G)
    rows1 = max(8, rows // (4 * threads))
    oracle.set_threads(1)
    try:
        dt1 = rate(0, rows1)
    finally:
        oracle.set_threads(threads)
    base = {
        "value": rows * E / dt,
        "unit": "Z entries/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"rows 0..{rows - 1} of the same {E}x{E} matrix ({rows * E} entries) in "
                  f"triangle-pair order, FP64 direct exp, {threads} threads, {dt:.1f} s",
        # point pairs the block evaluates: its test triangles x all triangles x Q^2
        "green_evals_per_s": np.unique(edges[:rows, 2:4]).size * F.shape[0] * Q * Q / dt,
        "table_mode": {"value": rows * E / dt_table, "seconds": dt_table, "tol": tol,
                       "table_over_direct": dt / dt_table},
        "one_thread": {"value": rows1 * E / dt1, "rows": rows1, "seconds": dt1},
        "lscpu": _lscpu(),
    }
    parity = None
    if sample is not None:
        flat, vals = sample
        t0 = time.perf_counter()
        ref = oracle.fill_entries(V, F, edges, k, Q, flat // E, flat % E)
        t_ref = time.perf_counter() - t0
        parity = {"sample": f"{flat.size} distinct flat indices of the {E}x{E} matrix "
                            f"(numpy default_rng(2), 1 %), FP64 oracle per entry, {t_ref:.1f} s"}
        for mode, z in vals.items():
            z = z.astype(np.complex128)
            nz_r, nz_i = ref.real != 0.0, ref.imag != 0.0
            er = np.abs(z.real - ref.real)[nz_r] / np.abs(ref.real[nz_r])
            ei = np.abs(z.imag - ref.imag)[nz_i] / np.abs(ref.imag[nz_i])
            parity[mode] = {
                "rel_frobenius": float(np.linalg.norm(z - ref) / np.linalg.norm(ref)),
                "re_rel_median": float(np.median(er)), "re_rel_p99": float(np.percentile(er, 99)),
                "im_rel_median": float(np.median(ei)), "im_rel_p99": float(np.percentile(ei, 99)),
            }
    return base, parity


def adjoint_timing(mf, steps):
    """dL/dV and dL/dk of L = Re sum conj(W) Z on the 7,680-unknown jittered
    sphere (k = 10, 6-point rule, W complex64 N(0,1))."""
    import torch

    from paper_1901_04162_amd import meshes

    wl = meshes.workload("ico4_grad")
    V, F, k, Q = wl["V"], wl["F"], wl["k"], wl["Q"]
    m = mf.Mesh(F, V.shape[0])
    E = m.n_edges
    g = torch.Generator(device="cuda").manual_seed(6)
    W = torch.complex(torch.randn(E, E, device="cuda", generator=g),
                      torch.randn(E, E, device="cuda", generator=g))
    Vd = torch.tensor(V, dtype=torch.float64, device="cuda")
    lo, hi = mf.r_range(m, Vd, Q)
    T = mf.build_tables(k, lo, hi, 1e-5)
    out = {"workload": f"icosphere 4 subdivisions, N(0, 0.01^2) vertex jitter ({F.shape[0]} "
                       f"triangles, {E} unknowns), k={k}, {Q}-point rule, W complex64"}
    for mode in ("table", "direct"):
        for _ in range(2):
            mf.fill_Z_backward(m, Vd, k, Q, mode, T, W)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            mf.fill_Z_backward(m, Vd, k, Q, mode, T, W)
        torch.cuda.synchronize()
        out[f"{mode}_ms"] = (time.perf_counter() - t0) / steps * 1e3
    for mode in ("table", "direct"):
        mf.fill_Z(m, Vd, k, Q, mode, T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            mf.fill_Z(m, Vd, k, Q, mode, T)
        torch.cuda.synchronize()
        out[f"forward_{mode}_ms"] = (time.perf_counter() - t0) / steps * 1e3
        out[f"{mode}_over_forward"] = out[f"{mode}_ms"] / out[f"forward_{mode}_ms"]
    return out


def sweep_timing(mf, steps, group=8, tol=1e-5):
    """Frequency sweep: three jittered icospheres (1,920 / 7,680 / 30,720
    unknowns) x 32 wavenumbers in [4, 20], 6-point rule, per-(mesh, k)
    tables.  The 96 items run as 4 batched launches of 3 meshes x 8
    wavenumbers, captured together in one CUDA graph; the groups share one
    set of complex64 outputs (64 GB), as a consumer would reuse them.  The
    first batch's creation runs the tile-shape tuner (the others reuse its
    choice); its timings are reported."""
    import torch

    from paper_1901_04162_amd import meshes

    wl = meshes.workload("sweep")
    Q, ks = wl["Q"], wl["k"]
    mesh_data = []
    for V, F in wl["meshes"]:
        m = mf.Mesh(F, V.shape[0])
        Vd = torch.tensor(V, dtype=torch.float64, device="cuda")
        lo, hi = mf.r_range(m, Vd, Q)
        Zs = [torch.empty((m.n_edges, m.n_edges), dtype=torch.complex64, device="cuda")
              for _ in range(group)]
        mesh_data.append((m, Vd, lo, hi, Zs))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tables = {(i, j): mf.build_tables(float(k), md[2], md[3], tol)
              for i, md in enumerate(mesh_data) for j, k in enumerate(ks)}
    torch.cuda.synchronize()
    t_tables = time.perf_counter() - t0
    batches = []
    for g0 in range(0, len(ks), group):
        items = [(md[0], md[1], float(ks[j]), tables[(i, j)], md[4][j - g0])
                 for i, md in enumerate(mesh_data) for j in range(g0, min(g0 + group, len(ks)))]
        batches.append(mf.Batch(items, Q, "table"))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for b in batches:
            b.fill()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for b in batches:
            b.fill()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    for md in mesh_data:
        mf.sync_status(md[0])
    entries = sum(md[0].n_edges ** 2 for md in mesh_data) * len(ks)
    shape, threads, tune_ms = batches[0].tuning()
    return {
        "workload": "3 jittered icospheres (1280/5120/20480 triangles) x 32 k in [4, 20] rad/m, "
                    "6-point rule, table tol 1e-5, complex64; 4 launches of 24 items in one graph",
        "items": len(mesh_data) * len(ks),
        "tuned_tile_shape": f"{shape} blocks",
        "tuned_threads": threads,
        "tuning_ms_eb512_eb768_eb1024_tb1024_tb512": tune_ms,
        "ms_per_sweep": dt * 1e3,
        "z_entries_per_s": entries / dt,
        "table_build_ms_per_sweep": t_tables * 1e3,
        "z_entries_per_s_with_tables": entries / (dt + t_tables),
    }


def near_timing(mf, mesh, V, Vd, k, Q, tables, steps):
    """Near-field fill (unknowns whose edge midpoints are within a quarter
    wavelength) of the same sphere, table and direct mode."""
    import torch

    r = 0.25 * 2 * 3.141592653589793 / k
    nf = mf.NearField(mesh, V, r)
    vals = torch.empty(nf.nnz, dtype=torch.complex64, device="cuda")
    out = {"r_near": r, "nnz": nf.nnz, "tiles": nf.n_tiles,
           "pairs_per_row": nf.nnz / mesh.n_edges}
    for mode in ("table", "direct"):
        for _ in range(2):
            nf.fill(Vd, k, Q, mode, tables, out=vals)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            nf.fill(Vd, k, Q, mode, tables, out=vals)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[f"{mode}_ms"] = dt * 1e3
        out[f"{mode}_near_entries_per_s"] = nf.nnz / dt
    return out


def mfie_timing(mf, mesh, Vd, k, Q, tables, steps):
    """The MFIE (K operator) on the same sphere: table and direct fill times
    (every entry computed: the operator is not symmetric) and the elementwise
    relative error of the table fill's real and imaginary parts against the
    direct fill (the paper's Fig. 3 measure), on a fixed sample of entries."""
    import numpy as np
    import torch

    E = mesh.n_edges
    out = {}
    Zs = {}
    for mode in ("table", "direct"):
        Z = torch.empty((E, E), dtype=torch.complex64, device="cuda")
        tab = tables if mode == "table" else None
        mf.fill_mfie(mesh, Vd, k, Q, mode, tab, out=Z)
        torch.cuda.synchronize()
        mf.set_timing(True)
        ph = []
        t0 = time.perf_counter()
        for _ in range(steps):
            mf.fill_mfie(mesh, Vd, k, Q, mode, tab, out=Z)
            ph.append(mf.timings(mesh))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        mf.set_timing(False)
        mf.sync_status(mesh)
        ph = np.array(ph)
        out[f"{mode}_ms"] = dt * 1e3
        out[f"{mode}_fill_ms"] = float(ph[:, 2].mean())
        out[f"{mode}_touching_fp64_ms"] = float(ph[:, 1].mean())
        out[f"{mode}_z_entries_per_s"] = E * E / dt
        Zs[mode] = Z
    out["table_over_direct"] = out["direct_ms"] / out["table_ms"]
    g = torch.Generator(device="cuda").manual_seed(5)
    idx = torch.randint(0, E * E, (1 << 20,), device="cuda", generator=g)
    zt = Zs["table"].view(-1)[idx].to(torch.complex128)
    zd = Zs["direct"].view(-1)[idx].to(torch.complex128)
    for part, f in (("real", torch.real), ("imag", torch.imag)):
        rel = (torch.abs(f(zt) - f(zd)) / torch.abs(f(zd)).clamp_min(1e-30)).cpu().numpy()
        out[f"rel_err_{part}_median"] = float(np.median(rel))
        out[f"rel_err_{part}_p99"] = float(np.percentile(rel, 99))
    out["max_abs_err_over_max_abs"] = float(
        (Zs["table"] - Zs["direct"]).abs().max() / Zs["direct"].abs().max())
    out["error_sample_entries"] = int(idx.numel())
    del Zs
    torch.cuda.empty_cache()
    return out


def angular_timing(mf, steps):
    """The paper's own inner scheme (angular transformation, n = 8 points on
    each source edge, FP64 integrals) on the 5,120-triangle sphere at k = 10
    with the 6-point rule: the linear Exp table (from r = 0, tol 1e-6) against
    computed exponentials; 3 n Q Exp(-jkr) per ordered triangle pair plus one
    per test point and source triangle."""
    import numpy as np
    import torch

    from paper_1901_04162_amd import meshes

    V, F = meshes.icosphere(4)
    k, Q, n = 10.0, 6, 8
    m = mf.Mesh(F, V.shape[0])
    E, T_ = m.n_edges, F.shape[0]
    Vd = torch.tensor(V, dtype=torch.float64, device="cuda")
    rmax = mf.angular_rmax(m, Vd, Q)
    tab = mf.build_exp_table(k, rmax, 1e-6)
    out = {"workload": "icosphere 4 subdivisions (5120 triangles, 7680 unknowns), k=10 rad/m, "
                       "6-point rule, 8 points per source edge, complex64 Z",
           "exp_table_samples": tab.n_exp, "r_max": rmax}
    exps = T_ * T_ * Q * (3 * n + 1)
    Zs = {}
    for mode in ("table", "direct"):
        Z = torch.empty((E, E), dtype=torch.complex64, device="cuda")
        mf.fill_angular(m, Vd, k, Q, n, mode, tab, out=Z)
        torch.cuda.synchronize()
        mf.set_timing(True)
        ph = []
        for _ in range(steps):
            mf.fill_angular(m, Vd, k, Q, n, mode, tab, out=Z)
            ph.append(mf.timings(m)[2])
        mf.set_timing(False)
        mf.sync_status(m)
        fill = float(np.mean(ph))
        out[f"{mode}_fill_ms"] = fill
        out[f"{mode}_z_entries_per_s"] = E * E / (fill * 1e-3)
        out[f"{mode}_exp_evals_per_s"] = exps / (fill * 1e-3)
        Zs[mode] = Z
    out["table_over_direct"] = out["direct_fill_ms"] / out["table_fill_ms"]
    out["max_abs_err_over_max_abs"] = float(
        (Zs["table"] - Zs["direct"]).abs().max() / Zs["direct"].abs().max())
    del Zs
    torch.cuda.empty_cache()
    return out


def scatter_timing(mf, steps):
    """The paper's scattering case: a PEC sphere of radius half a wavelength
    (ka = pi; icosphere with 4 subdivisions, 7,680 unknowns, 6-point rule)
    under an x-polarised plane wave along z: table fill (tol 1e-6),
    excitation, dense solve (library LU, complex128), far field in 361
    E-plane directions, with the EFIE and with the MFIE; the RCS of each table
    fill against that of its direct fill (the comparison with the Mie series
    is a test, not a benchmark)."""
    import numpy as np
    import torch

    from paper_1901_04162_amd import meshes

    V, F = meshes.icosphere(4)
    m = mf.Mesh(F, V.shape[0])
    k, Q = float(np.pi), 6
    Vd = torch.tensor(V, dtype=torch.float64, device="cuda")
    lo, hi = mf.r_range(m, Vd, Q)
    T = mf.build_tables(k, lo, hi, 1e-6)
    th = np.linspace(0.0, np.pi, 361)
    dirs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    out = {}

    def run(mode, op):
        fill = mf.fill_Z if op == "efie" else mf.fill_mfie
        rhs_fn = mf.rhs_planewave if op == "efie" else mf.rhs_planewave_mfie
        Z = fill(m, Vd, k, Q, mode, T if mode == "table" else None, dtype=torch.complex64)
        rhs = rhs_fn(m, Vd, k, Q, [0, 0, 1.0], [1.0, 0, 0], dtype=torch.complex128)
        I = torch.linalg.solve(Z.to(torch.complex128), rhs.unsqueeze(1)).squeeze(1)
        return mf.far_field(m, Vd, k, Q, I, dirs)[1]

    for op in ("efie", "mfie"):
        pre = "" if op == "efie" else "mfie_"
        for mode in ("table", "direct"):
            run(mode, op)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                sig = run(mode, op)
            torch.cuda.synchronize()
            out[f"{pre}{mode}_ms"] = (time.perf_counter() - t0) / steps * 1e3
            out[f"{pre}{mode}_rcs"] = sig.cpu().numpy()
        st, sd = out.pop(f"{pre}table_rcs"), out.pop(f"{pre}direct_rcs")
        out[f"{pre}rcs_rel_l2_table_vs_direct"] = float(np.linalg.norm(st - sd) /
                                                       np.linalg.norm(sd))
    out["workload"] = ("PEC sphere, radius half a wavelength (ka = pi), 5120 triangles, 7680 "
                       "unknowns, x-polarised plane wave along z; fill + excitation + solve + "
                       "far field, EFIE and MFIE")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--no-mfie", action="store_true")
    ap.add_argument("--no-angular", action="store_true")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--subdiv", type=int, default=5)
    ap.add_argument("--k", type=float, default=17.0)
    ap.add_argument("--q", type=int, default=7)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-near", action="store_true")
    ap.add_argument("--no-scatter", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 1 GiB buffer three times (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the fill would shard by row blocks of test edges, one block per GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1901_04162_amd as mf
    from paper_1901_04162_amd import meshes

    torch.cuda.set_device(0)
    if args.copy_probe:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": x.numel() * 4, "copies": 3}), flush=True)
        return
    V, F = meshes.icosphere(args.subdiv)
    k, Q = args.k, args.q
    mesh = mf.Mesh(F, V.shape[0])
    E = mesh.n_edges
    T_ = F.shape[0]
    n_touch = mesh.n_touching()
    evals = (T_ * T_ - n_touch) * Q * Q  # regular quadrature-point pairs, ordered (metric)
    evals_alg = evals // 2  # Z = Z^T: each unordered regular pair is needed once
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
            fill_ms.append(mf.timings(mesh) + mf.fill_timings(mesh))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        mf.set_timing(False)
        mf.sync_status(mesh)
        return wall / steps, np.array(fill_ms)

    # tile-shape tuner: times the table-fill kernels on this fill, keeps the fastest
    lo0, hi0 = mf.r_range(mesh, Vd, Q)
    _, tune_choice, tune_name, tune_ms = mf.tune_fill(mesh, Vd, k, Q, "table",
                                                      mf.build_tables(k, lo0, hi0, args.tol), out=Z)
    log(f"tuner: {tune_name} ({tune_ms} ms)")
    # uniform 1 % sample of the matrix for the parity of the timed fills
    flat = np.sort(np.random.default_rng(2).choice(E * E, size=E * E // 100, replace=False))
    flat_d = torch.tensor(flat, device="cuda")
    gathered = {}
    s_table, ph_table = timed(step_table, args.steps, args.warmup)
    gathered["table"] = Z.view(-1)[flat_d].cpu().numpy()
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
            # sampling density over [r_min, r_max] (Eq. (2) quotes 1e3-1e4 per wavelength)
            "green_samples_per_wavelength": T.n_green * (2 * math.pi / k) / (T.r_max - T.r_min),
            "exp_samples_per_wavelength": T.n_exp * (2 * math.pi / k) / (T.r_max - T.r_min),
            "fill_kernel": tune_name,
            "tuner_ms_tb1024_tb512_eb1024": tune_ms,
            "triangle_block_plan": dict(zip(("blocks", "tiles", "cut_edges", "rounds"),
                                            mesh.tb_plan())),
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
                      "range_and_tables": float(s_table * 1e3 - ph_table[:, :3].sum(1).mean()),
                      "regular_fill_tile_kernel": float(ph_table[:, 3].mean()),
                      "regular_fill_cut_edge_fixup": float(ph_table[:, 4].mean())},
    }
    if not args.no_direct:
        # the same tuner on the direct fill (its own cache key), then the timing
        _, _, tune_name_d, tune_ms_d = mf.tune_fill(mesh, Vd, k, Q, "direct", None, out=Z)
        log(f"tuner (direct): {tune_name_d} ({tune_ms_d} ms)")
        s_direct, ph_direct = timed(step_direct, args.steps, args.warmup)
        gathered["direct"] = Z.view(-1)[flat_d].cpu().numpy()
        log(f"direct step {s_direct*1e3:.2f} ms; phases {ph_direct.mean(0).round(3).tolist()}")
        out["direct"] = {
            "ms_per_step": s_direct * 1e3,
            "z_entries_per_s": E * E / s_direct,
            "green_evals_per_s": evals / s_direct,
            "regular_fill_ms": float(ph_direct[:, 2].mean()),
            "regular_fill_tile_kernel_ms": float(ph_direct[:, 3].mean()),
            "regular_fill_cut_edge_fixup_ms": float(ph_direct[:, 4].mean()),
            "fill_kernel": tune_name_d,
            "tuner_ms_tb1024_tb512_eb1024": tune_ms_d,
        }
        out["table_over_direct"] = s_direct / s_table
        out["table_over_direct_fill_only"] = float(ph_direct[:, 2].mean() / ph_table[:, 2].mean())
    # roofline of the dominant kernel: the tile kernel of the regular fill
    # (k_fill_tb on the triangle-block plan; the cut-edge fix-up after it is
    # HBM-bound and reported beside it)
    tile_s = float(ph_table[:, 3].mean()) * 1e-3
    fix_s = float(ph_table[:, 4].mean()) * 1e-3
    achieved = FLOPS_PER_EVAL * evals_alg / tile_s / 1e12
    traffic, fix_traffic = _traffic()
    tb = fix_s > 0.0
    out["roofline"] = {
        "bound": "alu",
        "kernel": "k_fill_tb (table mode, triangle blocks)" if tb else "k_fill (table mode, edge blocks)",
        "achieved": achieved,
        "peak": PEAK_FP32,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32,
        "traffic": traffic if tb else None,
        "flops_per_launch": FLOPS_PER_EVAL * evals_alg,
        "launch_ms": tile_s * 1e3,
    }
    if tb:
        out["cut_edge_fixup"] = {
            "kernel": "k_cut_fix",
            "ms": fix_s * 1e3,
            "cut_edges": mesh.tb_plan()[2],
            "hbm_bytes": fix_traffic,
            "hbm_tb_per_s": fix_traffic / fix_s / 1e12 if fix_traffic else None,
        }
    del Z, flat_d
    torch.cuda.empty_cache()
    if not args.no_mfie:
        log("mfie ...")
        out["mfie"] = mfie_timing(mf, mesh, Vd, k, Q, T, args.steps)
    if not args.no_angular:
        log("angular transformation ...")
        out["angular"] = angular_timing(mf, max(1, min(args.steps, 3)))
    if not args.no_near:
        log("near field ...")
        out["near_field"] = near_timing(mf, mesh, V, Vd, k, Q, T, args.steps)
    if not args.no_adjoint:
        log("adjoint ...")
        out["adjoint"] = adjoint_timing(mf, args.steps)
        torch.cuda.empty_cache()
    if not args.no_scatter:
        log("scattering ...")
        out["scatter"] = scatter_timing(mf, max(1, min(args.steps, 3)))
        torch.cuda.empty_cache()
    if not args.no_sweep:
        log("sweep ...")
        out["sweep"] = sweep_timing(mf, max(1, min(args.steps, 3)))
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"], out["rel_err"] = cpu_baseline(V, F, mesh.edges(), k, Q, args.tol,
                                                           args.cpu_seconds, (flat, gathered))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
