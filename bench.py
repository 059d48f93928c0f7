"""Benchmark: fast direct solve of the tensor-product nth-order FEM Poisson system.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = one full solve (forward transforms on every axis, division,
inverse transforms on every axis; plus the float64 refinement passes in the
float32+refine mode) of one right-hand side already resident in HBM.  Prints
one JSON line.  Only one GPU is supported: the transforms of one problem run
on one device (a multi-GPU slab decomposition is described in the design
notes but not built).
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1701_03967_amd import inputs  # noqa: E402

PEAK_HBM_GBS = 8000.0
# The paper's 2D n=9, K=1024 solve: "less than 2 min" for 9215^2 unknowns on a laptop
PAPER_UNKNOWNS_PER_S = {"c3_2d_n9_k1024": 9215 ** 2 / 120.0, "c4_3d_n9_k64": 575 ** 3 / 900.0}
METRIC = "solve time & unknowns/s, n=9 2D/3D; FP32+refine vs FP64 at rel err ≤1e-10"


def kernel_bytes(name: str, size: int, N: int, n0: int = 9) -> float:
    """Algorithmic HBM bytes of one launch of a named kernel (one read and one
    write of every array it touches)."""
    t = 4 if "32" in name.split("_")[0] else 8
    if name.startswith("transpose"):
        return size * 2 * t
    if name.startswith("apply"):
        # operator passes, first (last axis) .. last (axis 0): the first reads
        # u and writes two products, the middle ones (3D) read two and write
        # two, the last reads two and f (or r) and writes r; double-double
        # passes carry hi and lo planes (16 bytes per value), plain float64
        # passes one (incremental residual r -= A c: the last pass reads r)
        dd = not name.startswith("apply64")
        ax = int(name.rsplit("_ax", 1)[1].rstrip("t"))
        v = 16 if dd else 8
        if N == 1:
            return size * 24.0
        if ax == N - 1:
            return size * (8.0 + 2 * v)
        if ax > 0:
            return size * 4.0 * v
        return size * (2 * v + 8.0 + 8.0)
    if name.startswith("resid3p"):
        # 3D plane pass: reads u (or the correction), writes the two products
        # (double-double: hi and lo planes)
        return size * (40.0 if name.startswith("resid3pdd") else 24.0)
    if name.startswith("resid2"):
        # fused 2D residual: reads u (or the correction) and f (or r),
        # writes r
        return size * 24.0
    if name.startswith("band"):
        # algorithm (b) along axis 0 (order n0).  One-sweep kernel: the first
        # sweep reads y and writes z and the node pivots, the second reads
        # them and writes x.  Three-kernel form: cond reads y and writes the
        # node right-hand sides (1/n0 of the array), nodes moves the node
        # values through the elimination (read g, write g' and the pivot,
        # read both, write x), back reads y and the node values and writes
        # x.  Tiled kernel (short lines): y read once, x written once.
        if name.startswith("bandcond"):
            return size * (8.0 + 8.0 / n0)
        if name.startswith("bandback"):
            return size * (16.0 + 8.0 / n0)
        if name.startswith("bandtile"):
            return size * 16.0
        if name.startswith("bandnodes"):
            return size * 48.0 / n0
        return size * (32 + 16.0 / n0)
    last = N - 1
    ax_s = name.rsplit("_ax", 1)[1]
    ax = int(ax_s.rstrip("t"))
    # the update passes of the refinement read u and write u (float64); with
    # N >= 2 they also store the correction (float64)
    upd = (16.0 if N >= 2 else 8.0) if "upd" in name else 0.0
    if name.startswith("fwd"):
        rd = 8 if ax == last else t
        return size * (rd + t)
    if name.startswith("mid"):
        rd = 8 if N == 1 else t
        wr = 8 if N == 1 else t
        return size * (rd + wr + upd)
    if name.startswith("inv"):
        wr = 8 if ax == last else t
        return size * (t + wr + upd)
    return 0.0


KERNEL_SOURCES = ("line.hip", "fft.h", "spectral.h", "device_common.h", "launch.h", "ops.hip", "api.cpp", "band.hip",
                  "long.hip", "batch.cpp")


def sources_sha256() -> str:
    """Hash of the kernel sources and their launch code: counter summaries
    taken on other sources no longer describe the kernels."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1701_03967_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiler_kernel_name(name: str, n: int, N: int, K: int) -> str:
    """Symbol of the kernel that a per-pass timing name refers to."""
    head = name.split("_ax")[0]
    if head.startswith("transpose"):
        return f"transpose_kernel<{'float' if head.endswith('32') else 'double'}>"
    for pre, sym in (("bandcond", "band_cond_kernel"), ("bandnodes", "band_nodes_kernel"),
                     ("bandback", "band_back_kernel"), ("bandtile", "band_tile_kernel"), ("band", "band_kernel")):
        if head.startswith(pre):
            # the tiled kernel also carries its lines per workgroup: match
            # the symbol's prefix
            return f"{sym}<{n}, " if pre == "bandtile" else f"{sym}<{n}>"
    if head.startswith("resid3p"):
        return f"resid3p_kernel<{n}, {'true' if head == 'resid3pdd' else 'false'}>"
    if head.startswith("resid2"):
        return f"resid2_kernel<{n}, {'true' if head == 'resid2dd' else 'false'}>"
    if head.startswith("apply"):
        dd = not head.startswith("apply64")
        ax = int(name.rsplit("_ax", 1)[1].rstrip("t"))
        lo = dd and ax != N - 1
        return f"apply_kernel<{n}, {'true' if lo else 'false'}, {'true' if dd else 'false'}>"
    dtype = "double" if head.endswith("64") else "float"
    mode = 0 if head.startswith("fwd") else (1 if head.startswith("inv") else 2)
    upd = "true" if "upd" in head else "false"
    ax = name.rsplit("_ax", 1)[1]
    contiguous = ax.endswith("t") or int(ax.rstrip("t")) == N - 1
    # the kernel object: 0 powers of two, 1 mixed radix (prime factors <= 7), 2 Bluestein
    kind = 0 if K & (K - 1) == 0 else (1 if smooth7(K) else 2)
    return f"line_kernel<{dtype}, {n}, {mode}, {upd}, {'false' if contiguous else 'true'}, {kind}>"


def smooth7(K: int) -> bool:
    for p in (2, 3, 5, 7):
        while K % p == 0:
            K //= p
    return K == 1


def measured_traffic(workload: str, kernel: str, mode: str = ""):
    """HBM bytes per dispatch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size) of the
    mode's own runs (one kernel symbol can serve several modes with other
    layouts), else of the workload's, or None when there is none or the
    kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{mode}.txt")
    if not mode or not os.path.exists(path):
        path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    sha, rows = None, {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("sources_sha256:"):
                sha = line.split(":", 1)[1].strip()
            elif line.startswith("kernel:"):
                parts = [x.strip() for x in line[len("kernel:"):].split("|")]
                kv = dict(x.split("=", 1) for x in parts[1:])
                rows[parts[0]] = float(kv["bytes"])
    if sha != sources_sha256():
        return None
    for k, v in rows.items():
        if kernel in k:
            return v
    return None


def copy_calibration(torch, nbytes: int):
    """One plain device-to-device copy of nbytes (the counters' scale)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def time_mode(fm, torch, prob, f, precision, steps, warmup, timing=True, tune=False, graph=False):
    """Mean and median of `steps` solves (direct launches, events per step,
    no per-kernel instrumentation), then per-kernel times from a separate
    instrumented run, and with `graph` the mean of graph replays of one
    captured solve.  Returns (plan, u, ms, kernels, stats, extra)."""
    algorithm = "a"
    if precision.endswith("_b"):
        precision, algorithm = precision[:-2], "b"
    plan = fm.Plan(prob.K, prob.n, prob.diff, prob.react, precision=precision,
                   max_iter=3 if precision == "fp32_refine" else 0, tol=1e-12, algorithm=algorithm)
    if tune and prob.N >= 2:
        plan.tune()  # measured line-pass parameters, before the untimed warm-up
    u = torch.empty_like(f)
    for _ in range(warmup):
        plan.solve(f, u)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        plan.solve(f, u)
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    ms = ev[0].elapsed_time(ev[steps]) / steps
    extra = {"median_ms": float(np.median(per)), "min_ms": float(np.min(per))}
    st = plan.stats()
    kt = {}
    if timing:
        plan.get_timing()
        plan.set_timing(True)
        for _ in range(min(steps, 10)):
            plan.solve(f, u)
        torch.cuda.synchronize()
        kt = plan.get_timing()
        plan.set_timing(False)
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            plan.solve(f, u)
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.solve(f, u)
        g.replay()
        torch.cuda.synchronize()
        gev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        gev[0].record()
        for i in range(steps):
            g.replay()
            gev[i + 1].record()
        torch.cuda.synchronize()
        gper = [gev[i].elapsed_time(gev[i + 1]) for i in range(steps)]
        extra["graph_ms"] = gev[0].elapsed_time(gev[steps]) / steps
        extra["graph_median_ms"] = float(np.median(gper))
        del g
    return plan, u, ms, kt, st, extra


def golden_path(workload: str) -> str:
    return os.path.join(ROOT, "tests", "golden", f"fullsize_{workload}.txt")


def load_golden(workload: str):
    """The oracle's stored solution of a full-size workload (written by
    tests/golden/make_fullsize.py from the CPU oracle): global norms and
    projections, sampled indices and values, and the refinement corrections
    the oracle's solve computed.  None if there is no fixture."""
    path = golden_path(workload)
    if not os.path.exists(path):
        return None
    glob, idx, val, corr = {}, [], [], None
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("#"):
                if "relative corrections" in line:
                    corr = len(re.findall(r"\d\.\d+e[-+]\d+", line.split("relative corrections", 1)[1]))
                continue
            if not line:
                continue
            a, b = line.split()
            if a in ("l2", "max", "sum") or a.startswith("proj"):
                glob[a] = float(b)
            else:
                idx.append(int(a))
                val.append(float(b))
    return {"glob": glob, "idx": np.array(idx, dtype=np.int64), "val": np.array(val), "corrections": corr}


class OracleCheck:
    """Relative errors of a device solution against the oracle's stored one:
    over the stored samples (l2), and the largest difference of the inner
    products with the seeded sign vectors relative to ||u|| (any error of the
    solution moves them by about its l2 norm, wherever it sits)."""

    def __init__(self, torch, workload: str, shape):
        self.g = load_golden(workload)
        self.torch = torch
        self.probes = []
        if self.g is not None:
            self.idx = torch.from_numpy(self.g["idx"]).cuda()
            for i in range(inputs.NPROBE):
                if f"proj{i}" in self.g["glob"]:
                    self.probes.append((self.g["glob"][f"proj{i}"],
                                        torch.from_numpy(inputs.probe_vector(shape, i)).cuda().view(-1)))

    def __call__(self, u):
        if self.g is None:
            return None
        flat = u.view(-1)
        got = flat[self.idx].cpu().numpy()
        ref = self.g["val"]
        out = {"samples": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}
        l2 = self.g["glob"]["l2"]
        if self.probes:
            out["proj"] = float(max(abs(float(self.torch.dot(w, flat)) - v) for v, w in self.probes) / l2)
        out["max"] = max(out.values())
        return out


def cpu_baseline(prob, workload: str):
    """The CPU oracle's solve, timed on the host cores (a bounded sample).

    The oracle solves by dense per-axis eigenvectors: u = S (S^T f / den)
    with the Kronecker factors applied as mode products (dense GEMMs), then
    refinement with the residual of the exact operator in extended precision.
    Timed here with the oracle's own functions: one whole apply_inverse at
    the full size (its GEMM cost does not depend on the values, so random
    factors stand in for the eigenvectors), and the extended-precision
    residual on a block of lines at full line length, scaled to the array.
    The solve is one apply_inverse plus, per refinement correction the
    oracle computed for this workload (its stored history), one residual and
    one apply_inverse.  The eigendecomposition (plan work, which the paper
    also leaves out of its timings) is reported separately: timed at the
    full size when the axis has at most 2000 dofs, else on the same order
    with K/4 elements and scaled by the cube of the size ratio.
    """
    from oracle import fem1d, solve as osolve
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        blas = os.cpu_count() or 1
    shape = prob.shape
    size = prob.size
    g = inputs.generator(0)
    f = g.standard_normal(shape)
    # one apply_inverse at full size
    s = osolve.EigenSolver.__new__(osolve.EigenSolver)
    s.S = [g.standard_normal((m, m)) for m in shape]
    s.den = np.ones(shape)
    t0 = time.perf_counter()
    s.apply_inverse(f)
    t_inv = time.perf_counter() - t0
    del s
    # extended-precision residual on a block of lines along axis 0
    rows = max(1, min(shape[0], int(4000000 // max(1, size // shape[0]))))
    Kb = (max(1, (rows + 1) // prob.n),) + tuple(prob.K[1:])
    blk = np.ascontiguousarray(f[: prob.n * Kb[0] - 1])
    t0 = time.perf_counter()
    osolve.apply_A(blk, prob.n, Kb, prob.diff, prob.react, extended=True)
    t_res = (time.perf_counter() - t0) * size / blk.size
    del f, blk
    gold = load_golden(workload)
    ncorr = gold["corrections"] if gold and gold["corrections"] else 3
    total = (1 + ncorr) * t_inv + ncorr * t_res
    # eigendecomposition of one axis
    M = shape[0]
    Ke = prob.K[0] if M <= 2000 else max(2, prob.K[0] // 4)
    t0 = time.perf_counter()
    fem1d.dense_eigen(prob.n, Ke)
    t_eig = (time.perf_counter() - t0) * ((prob.n * prob.K[0] - 1) / (prob.n * Ke - 1)) ** 3
    axes = len(set(prob.K))
    return {"value": size / total, "unit": "unknowns/s", "cores": int(blas), "kind": "oracle",
            "host_cpus": os.cpu_count(),
            "sample": (f"dense-eigen oracle solve: one apply_inverse timed at full size ({t_inv:.2f} s), the "
                       f"extended-precision residual timed on {blk_rows(prob, Kb)} of {shape[0]} lines along "
                       f"axis 0 and scaled ({t_res:.2f} s per residual); {ncorr} refinement corrections "
                       f"(the oracle's history for this workload); eigendecomposition excluded"),
            "seconds_per_solve": total, "apply_inverse_s": t_inv, "residual_s": t_res,
            "refinement_corrections": ncorr,
            "eigendecomposition_s": t_eig * axes,
            "eigendecomposition": (f"{axes} distinct axis pencil(s) of size {M}: "
                                   + ("timed" if Ke == prob.K[0] else
                                      f"timed at K={Ke} (size {prob.n * Ke - 1}) and scaled by the size ratio cubed"))}


def blk_rows(prob, Kb):
    return prob.n * Kb[0] - 1


def run_batch(args, torch, fm):
    """The batched heat-step workload: 512 independent 2D problems (n in 2..8,
    K per axis in 32..512, diff in [0.5, 2], react = 1/tau = 1000, 1..8
    right-hand sides), float32 transforms with float64 refinement (or, with
    --batch-precision fp64, float64 transforms), solved in one graph launch;
    line-pass parameters tuned on the first solve.
    Right-hand sides: N(0,1), drawn on the device per problem from a seeded
    generator (the problem parameters come from the seeded workload draw)."""
    draw = inputs.draw_batch(count=args.batch_count)
    prec = args.batch_precision
    probs = [dict(K=p.K, n=p.n, diff=p.diff, react=p.react, precision=prec,
                  max_iter=args.batch_iters if prec == "fp32_refine" else 0, tol=1e-12, nrhs=p.nrhs)
             for p in draw.problems]
    total = sum(p.nrhs * p.size for p in draw.problems)
    t0 = time.perf_counter()
    b = fm.Batch(probs, tune=not args.no_tune)
    t_plan = time.perf_counter() - t0
    fs, us = [], []
    for i, p in enumerate(draw.problems):
        g = torch.Generator(device="cuda")
        g.manual_seed(draw.seeds[i])
        shape = ((p.nrhs,) if p.nrhs > 1 else ()) + p.shape
        fs.append(torch.randn(shape, generator=g, dtype=torch.float64, device="cuda"))
        us.append(torch.empty_like(fs[-1]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.solve(fs, us)  # records, tunes, captures the graph, then runs it
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    print(f"[bench] batch: {len(probs)} problems, {total} unknowns, plan {t_plan:.1f}s, "
          f"first solve (record + tune + capture) {t_first:.1f}s", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        b.solve(fs, us)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        b.solve(fs, us)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    its = [b.stats(i)["iterations"] for i in range(len(probs))]
    conv = sum(b.stats(i)["converged"] for i in range(len(probs)))
    line = {
        "metric": "batched solve: unknowns/s over all problems and right-hand sides",
        "value": total / (ms * 1e-3),
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == "fp32_refine" else ("f64" if prec == "fp64" else "f32"),
        "data": "synthetic",
        "config": {"workload": f"c5_batch_{len(probs)}_2d_heat_step", "problems": len(probs),
                   "unknowns": total, "react": draw.problems[0].react, "precision": prec,
                   "max_iter": args.batch_iters if prec == "fp32_refine" else 0, "tuned": not args.no_tune},
        "plan_s": t_plan, "first_solve_s": t_first,
        "refinement": {"iterations_min": min(its), "iterations_max": max(its), "converged": conv},
        "workspace_bytes": b.workspace_bytes(),
    }
    # HBM roofline of the whole batch on the per-dof pass model of a 2D
    # solve: float64 3 passes x 16 B; float32 12 + 8 + 12 B; each refinement
    # step 20 + 8 + 20 B (residual, float32 chain, update), at the mean
    # number of steps taken
    per = {"fp64": 48.0, "fp32": 32.0}.get(prec, 32.0 + 48.0 * float(np.mean(its)))
    gbs = line["value"] * per / 1e9
    line["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None,
                        "model_bytes_per_unknown": per, "kernel": "whole batch"}
    if getattr(args, "quiet", False):
        return line
    print(json.dumps(line))


def run_long2d(args, torch, fm):
    """2D solves with both axes longer than one LDS tile (n = 9, K per axis
    2048, 4096 and 11000: 3.4e8, 1.36e9 and 9.8e9 unknowns, the last filling
    most of the 288 GB of HBM: f, u and the plan's transposed copy at 78.4 GB
    each), float64 by algorithm (a) through the multi-pass long-line
    transforms: the element-count scaling beyond the C3 size.  Synthetic
    N(0,1) load, resident in HBM; mean of the timed solves and per-kernel
    times."""
    n = 9
    rows = []
    for Kd in (2048, 4096, 11000):
        plan = fm.Plan((Kd, Kd), n, (1.0, 1.0), 0.0)
        g = torch.Generator(device="cuda")
        g.manual_seed(Kd)
        f = torch.randn(plan.shape, generator=g, dtype=torch.float64, device="cuda")
        u = torch.empty_like(f)
        for _ in range(args.warmup):
            plan.solve(f, u)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        steps = max(3, args.steps // 5)
        e0.record()
        for _ in range(steps):
            plan.solve(f, u)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        plan.get_timing()
        plan.set_timing(True)
        plan.solve(f, u)
        torch.cuda.synchronize()
        kt = {k: v[0] for k, v in plan.get_timing().items()}
        plan.set_timing(False)
        st = plan.stats()
        # finiteness in blocks of rows (no full-size temporary)
        finite = all(bool(torch.isfinite(u[r0:r0 + 4096]).all().item()) for r0 in range(0, u.shape[0], 4096))
        rows.append({"K": [Kd, Kd], "unknowns": f.numel(), "ms": ms, "unknowns_per_s": f.numel() / (ms * 1e-3),
                     "finite": finite, "stop": st["stop"], "kernels_ms": kt,
                     "workspace_bytes": plan.workspace_bytes()})
        print(f"[bench] long2d K={Kd}: {ms:.2f} ms/solve ({f.numel()} unknowns)", file=sys.stderr, flush=True)
        del plan, f, u
        torch.cuda.empty_cache()
    line = {
        "metric": "2D solve time & unknowns/s beyond one LDS tile per axis, n=9, float64",
        "value": rows[-1]["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": max(3, args.steps // 5),
        "warmup": args.warmup,
        "ms_per_step": rows[-1]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "long2d_n9", "n": 9, "value": "the largest K"},
        "per_K": rows,
    }
    print(json.dumps(line))


def run_heat(args, torch, fm):
    """Implicit Euler time stepping on the C3 mesh (2D, n = 9, K = 1024,
    diff (1, 1)) with tau = 1e-3 (react = 1000, the batched workload's heat
    step): u^0 and the load drawn N(0,1) on the device from seeded
    generators; each step is one double-double mass apply and one solve with
    the reused plan (float64).  Value: unknowns advanced per second."""
    prob = inputs.WORKLOADS["c3_2d_n9_k1024"].problem
    react = 1000.0
    plan = fm.Plan(prob.K, prob.n, prob.diff, react, precision=args.heat_precision,
                   max_iter=3 if args.heat_precision == "fp32_refine" else 0, tol=1e-12)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    u = torch.randn(prob.shape, generator=g, dtype=torch.float64, device="cuda")
    F = torch.randn(prob.shape, generator=g, dtype=torch.float64, device="cuda")
    work = torch.empty_like(u)
    nsteps = args.heat_steps
    plan.implicit_euler(u, args.warmup, F=F, work=work)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.implicit_euler(u, nsteps, F=F, work=work)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    line = {
        "metric": "implicit Euler heat steps: unknowns advanced per second",
        "value": prob.size * nsteps / (ms * 1e-3),
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.heat_precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "heat_c3_2d_n9_k1024_tau1e-3", "unknowns": prob.size, "react": react,
                   "time_steps_per_step": nsteps, "precision": args.heat_precision},
        "ms_per_time_step": ms / nsteps,
    }
    print(json.dumps(line))


TRANSFORM_K = {"pow2": (32, 64, 128, 256, 512, 1024), "prime": (31, 61, 127, 257, 509, 1021),
               "composite": (48, 96, 200, 384, 600, 1000),
               "long": (1 << 11, 1 << 12, 1 << 14, 1 << 16, 1 << 18, 1 << 20),
               # one prime and one composite per octave up to 2^20 (the composites drawn once at
               # random, fixed here)
               "long_prime": (1031, 2053, 4099, 8209, 16411, 32771, 65537, 131101, 262147, 524309, 1048573),
               "long_composite": (1662, 2308, 5481, 11099, 32551, 60695, 89354, 221294, 319564, 543195)}


def run_transform1d(args, torch, fm):
    """1D FC_n (forward) and F_n (inverse) transforms, n = 5, along the
    contiguous axis of a 3D array of about 2^26 dofs (the lines are the other
    two axes), for element counts that are powers of two, primes and
    composites (the latter two through chirp-z DFTs); float64.  Long lines
    (1024 < K <= 2^20: powers of two, primes and composites): one-axis plans
    whose right-hand sides are the lines, through the multi-pass four-step
    transforms (Bluestein's for K not a power of two), with the mean time of
    each of their kernels.  Per K: the mean time of one transform of all
    lines, dofs/s and GB/s (one read and one write of 8 bytes per dof)."""
    n = 5
    rows = []
    kinds = [k.strip() for k in args.transform_kinds.split(",") if k.strip()]
    for kind in kinds:
        for K in TRANSFORM_K[kind]:
            M = n * K - 1
            lines = max(1, (1 << 26) // M)
            long_line = kind.startswith("long")
            if long_line:
                plan = fm.Plan((K,), n, (1.0,), 0.0, nrhs=lines)
                axis, nl = 0, lines
            else:
                k0 = max(2, min(1024, int(round(np.sqrt(lines) / n))))
                k1 = max(2, min(1024, int(round(lines / (n * k0 - 1) / n))))
                plan = fm.Plan((k0, k1, K), n, (1.0, 1.0, 1.0), 0.0)
                axis, nl = 2, plan.shape[0] * plan.shape[1]
            shape = (lines, M) if long_line else plan.shape
            g = torch.Generator(device="cuda")
            g.manual_seed(K)
            x = torch.randn(shape, generator=g, dtype=torch.float64, device="cuda")
            y = torch.empty_like(x)
            rec = {"kind": kind, "K": K, "lines": nl, "dofs": x.numel()}
            for name, d in (("fc_n", +1), ("f_n", -1)):
                for _ in range(args.warmup):
                    plan.debug_transform(axis, d, x, y)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(args.steps):
                    plan.debug_transform(axis, d, x, y)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                rec[name] = {"ms": ms, "dofs_per_s": x.numel() / (ms * 1e-3),
                             "GB_per_s": 16 * x.numel() / (ms * 1e-3) / 1e9}
                if long_line:
                    plan.get_timing()
                    plan.set_timing(True)
                    for _ in range(min(args.steps, 5)):
                        plan.debug_transform(axis, d, x, y)
                    torch.cuda.synchronize()
                    rec[name]["kernels_ms"] = {k: v[0] for k, v in plan.get_timing().items()}
                    plan.set_timing(False)
            rows.append(rec)
            print(f"[bench] transform1d {kind} K={K}: fc_n {rec['fc_n']['ms']:.3f} ms, "
                  f"f_n {rec['f_n']['ms']:.3f} ms ({rec['dofs']} dofs)", file=sys.stderr, flush=True)
            if long_line:
                for name in ("fc_n", "f_n"):
                    ks = ", ".join(f"{k} {v:.3f}" for k, v in rec[name]["kernels_ms"].items())
                    print(f"[bench]   {name} kernels (ms): {ks}", file=sys.stderr, flush=True)
            del plan, x, y
    fwd = [r["fc_n"]["dofs_per_s"] for r in rows if r["kind"] == "pow2"] or [r["fc_n"]["dofs_per_s"] for r in rows]
    line = {
        "metric": "1D FC_n / F_n transform throughput, n=5 (dofs/s)",
        "value": float(np.exp(np.mean(np.log(fwd)))),
        "unit": "dofs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean([r["fc_n"]["ms"] for r in rows])),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "transform1d_n5", "n": 5, "value": "geometric mean of the forward "
                   "transform over the power-of-two K up to 1024 (all K measured when those are not)"},
        "per_K": rows,
    }
    print(json.dumps(line))


def summarize_stats(d: str, title: str, cmd: str, out: str):
    """profiles/kernel_stats_<name>.txt from the kernel_stats.csv of a
    rocprofv3 --kernel-trace --stats run in directory d, longest total first."""
    import csv
    import glob
    fn = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = []
    with open(fn) as fh:
        for r in csv.DictReader(fh):
            rows.append((float(r["TotalDurationNs"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                         float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"]), r["Name"]))
    rows.sort(reverse=True)
    lines = [f"# rocprofv3 --kernel-trace --stats summary (kernel_stats.csv), MI355X (gfx950): {title}",
             f"# command: (from the repository root, TMPDIR=/tmp) {cmd}",
             f"# summary: python bench.py summarize-stats <output dir> <title> <command> <this file>",
             f"# kernel sources sha256: {sources_sha256()}",
             " calls     avg_us     min_us     max_us    pct  kernel"]
    for _, calls, avg, mn, mx, pct, name in rows:
        if len(name) > 160:  # library kernels with long template names
            name = name[:157] + "..."
        lines.append(f"{calls:6d} {avg:10.1f} {mn:10.1f} {mx:10.1f} {pct:6.2f}  {name}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines[:30]))


def summarize_traffic(workload: str, fetch_dir: str, write_dir: str, nbytes: str, fetch_cmd: str,
                      write_cmd: str, out: str):
    """profiles/traffic_<workload>.txt from two rocprofv3 --pmc runs of the
    same bench command (FETCH_SIZE, WRITE_SIZE), scaled by what the counters
    read for the calibration copy (the largest device copy of the run, a
    plain copy of nbytes bytes)."""
    import csv
    import glob
    from collections import defaultdict
    nbytes = int(nbytes)

    def read(d, counter):
        per = defaultdict(list)
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(fn) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] == counter:
                        per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return per

    fe, wr = read(fetch_dir, "FETCH_SIZE"), read(write_dir, "WRITE_SIZE")
    copy_f = max(v for k, vs in fe.items() if "copyBuffer" in k for v in vs)
    copy_w = max(v for k, vs in wr.items() if "copyBuffer" in k for v in vs)
    ff, fw = nbytes / 1024.0 / copy_f, nbytes / 1024.0 / copy_w
    lines = [f"# HBM traffic per dispatch, workload {workload}, MI355X (gfx950), rocprofv3 --pmc",
             f"# fetch pass: (from the repository root, TMPDIR=/tmp) {fetch_cmd}",
             f"# write pass: (from the repository root, TMPDIR=/tmp) {write_cmd}",
             f"# summary: python bench.py summarize-traffic {workload} <fetch dir> <write dir> {nbytes} "
             "<fetch command> <write command> <this file>",
             f"# scale: a plain device copy of {nbytes} bytes read FETCH_SIZE {copy_f:.1f} KiB and WRITE_SIZE "
             f"{copy_w:.1f} KiB; factors fetch x{ff:.4f}, write x{fw:.4f}",
             "# bytes = (FETCH_SIZE * fetch factor + WRITE_SIZE * write factor) * 1024, mean over dispatches",
             f"sources_sha256: {sources_sha256()}"]
    rows = []
    for k in fe:
        if "fftfem::" not in k or k not in wr:
            continue
        f = sum(fe[k]) / len(fe[k]) * ff * 1024
        w = sum(wr[k]) / len(wr[k]) * fw * 1024
        rows.append((f + w, f"kernel: {k} | dispatches={len(fe[k])} | fetch_bytes={f:.4e} | "
                            f"write_bytes={w:.4e} | bytes={f + w:.6e}"))
    lines += [r for _, r in sorted(rows, reverse=True)]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_replay(d: str, cmd: str, out: str):
    """profiles/<name>.txt from the kernel trace of a run that replays one
    captured graph several times (the batched workload): the last three
    replays (the periodic tail of the trace), each one's wall time against the
    union of its kernels' intervals, the idle gaps between kernels, and the
    kernels taking most of a replay."""
    import csv
    import glob
    from collections import defaultdict
    rows = []
    for fn in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        with open(fn) as fh:
            for r in csv.DictReader(fh):
                if "fftfem::" in r["Kernel_Name"]:
                    rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    names = [r[2] for r in rows]
    n = len(names)
    period = None
    for cand in range(100, n // 3 + 1):
        if names[-cand:] == names[-2 * cand:-cand] == names[-3 * cand:-2 * cand]:
            period = cand
            break
    lines = ["# graph replays of the batched workload: kernel busy time against wall time, MI355X (gfx950)",
             f"# command: (from the repository root, TMPDIR=/tmp) {cmd}",
             "# summary: python bench.py summarize-replay <output dir> <command> <this file>",
             f"# kernel sources sha256: {sources_sha256()}",
             f"fftfem kernels in the trace: {n}"]
    if period is None:
        lines.append("no periodic tail (three identical replays) found")
    for rep in range(3 if period else 0):
        seg = rows[n - (rep + 1) * period: n - rep * period]
        t0, t1 = seg[0][0], max(e for _, e, _ in seg)
        busy, cs, ce = 0, None, None
        for st, en, _ in seg:
            if ce is None or st > ce:
                if ce is not None:
                    busy += ce - cs
                cs, ce = st, en
            else:
                ce = max(ce, en)
        busy += ce - cs
        lines.append(f"replay -{rep + 1}: launches {period}, wall {(t1 - t0) / 1e6:.3f} ms, busy (union of kernel "
                     f"intervals) {busy / 1e6:.3f} ms ({busy / (t1 - t0):.4f} of wall)")
        if rep == 0:
            last, gaps = seg[0][1], []
            for st, en, _ in seg[1:]:
                gaps.append(max(0, st - last))
                last = max(last, en)
            gaps.sort()
            lines.append(f"  idle gaps between kernels: total {sum(gaps) / 1e6:.3f} ms, median "
                         f"{gaps[len(gaps) // 2] / 1e3:.2f} us, p90 {gaps[int(len(gaps) * 0.9)] / 1e3:.2f} us, "
                         f"max {gaps[-1] / 1e3:.2f} us")
            per = defaultdict(lambda: [0, 0])
            for st, en, nm in seg:
                per[nm][0] += en - st
                per[nm][1] += 1
            lines.append("  kernels by time in the replay (ms, launches):")
            for nm, (tt, c) in sorted(per.items(), key=lambda kv: -kv[1][0])[:20]:
                lines.append(f"    {tt / 1e6:9.3f} {c:5d}  {nm[:120]}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_counters(d: str, bench_json: str, title: str, cmd: str, out: str):
    """profiles/counters_<name>.txt from a rocprofv3 --pmc run of SQ
    counters (SQ_WAVES, SQ_INSTS_VALU, SQ_INSTS_LDS, SQ_WAIT_INST_LDS,
    SQ_WAVE_CYCLES, ...) in directory d: per kernel the mean over its
    dispatches, and, with the kernel's mean duration from a bench line on the
    same sources (bench_json; the mean over the modes that launch the kernel:
    an unprofiled run, since the profiler slows the kernels), VALU busy
    (VALU instructions x 4 cycles
    per wave64 instruction over 4 SIMDs x 256 CUs x the kernel's cycles at
    2.4 GHz), the LDS-wait share of the wave cycles, and the mean resident
    waves per CU (SQ_WAVE_CYCLES, counted in units of 4 cycles, over 256 x
    the kernel's cycles)."""
    import csv
    import glob
    from collections import defaultdict
    acc = defaultdict(lambda: defaultdict(list))
    for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(fn) as fh:
            for r in csv.DictReader(fh):
                try:
                    acc[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
                except (KeyError, ValueError):
                    continue
    # mean duration per kernel symbol over the modes that launch it
    durs = defaultdict(list)
    with open(bench_json) as fh:
        rec = json.loads([line for line in fh.read().splitlines() if line.startswith("{")][-1])
    cfg = rec["config"]
    for mode in rec.get("modes", {}).values():
        for nm, t in mode.get("kernels_ms", {}).items():
            durs[profiler_kernel_name(nm, cfg["n"], cfg["N"], cfg["K"][0])].append(t)
    ms = {sym: sum(v) / len(v) for sym, v in durs.items()}
    lines = [f"# rocprofv3 --pmc SQ counters, MI355X (gfx950): {title}",
             f"# command: (from the repository root, TMPDIR=/tmp) {cmd}",
             "# summary: python bench.py summarize-counters <output dir> <bench line of the same sources> <title> "
             "<command> <this file>",
             f"# kernel sources sha256: {sources_sha256()}",
             "# per kernel: mean over its dispatches of each counter; derived figures use the kernel's mean "
             "duration in the default bench run (no profiler), averaged over the modes that launch it",
             "kernel | ms | waves | VALU instr/wave | LDS instr/wave | VALU busy | LDS-wait share | waves/CU"]
    for name, cs in sorted(acc.items()):
        mean = {c: sum(v) / len(v) for c, v in cs.items()}
        t = next((v for sym, v in ms.items() if sym in name), None)
        waves = mean.get("SQ_WAVES", 0.0)
        row = [name[:110], f"{t:.3f}" if t else "-", f"{waves:.0f}"]
        row.append(f"{mean.get('SQ_INSTS_VALU', 0) / waves:.0f}" if waves else "-")
        row.append(f"{mean.get('SQ_INSTS_LDS', 0) / waves:.0f}" if waves else "-")
        if t and waves:
            cyc = t * 1e-3 * 2.4e9
            row.append(f"{mean.get('SQ_INSTS_VALU', 0) * 4 / (4 * 256 * cyc):.2f}")
            wc = mean.get("SQ_WAVE_CYCLES", 0.0)
            row.append(f"{mean.get('SQ_WAIT_INST_LDS', 0) / wc:.3f}" if wc else "-")
            row.append(f"{wc * 4 / (256 * cyc):.1f}")
        else:
            row += ["-", "-", "-"]
        lines.append(" | ".join(row))
    lines.append("# counter means")
    for name, cs in sorted(acc.items()):
        lines.append(f"kernel: {name[:140]}")
        for c, v in sorted(cs.items()):
            lines.append(f"    {c} mean={sum(v) / len(v):.6g} dispatches={len(v)}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines[:20]))


def main():
    if len(sys.argv) > 1 and sys.argv[1] in ("summarize-stats", "summarize-traffic", "summarize-replay",
                                             "summarize-counters"):
        # text summaries of rocprofv3 output for profiles/ (no GPU use)
        fn = {"summarize-stats": summarize_stats, "summarize-traffic": summarize_traffic,
              "summarize-replay": summarize_replay, "summarize-counters": summarize_counters}[sys.argv[1]]
        fn(*sys.argv[2:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3_2d_n9_k1024")
    ap.add_argument("--also", default="c4_3d_n9_k64", help="second workload ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload in the default line")
    ap.add_argument("--transform-kinds", default="pow2,prime,composite,long,long_prime,long_composite",
                    help="element-count families of the transform1d workload")
    ap.add_argument("--modes", default="fp64,fp32,fp32_refine,fp64_b",
                    help="fp64, fp32, fp32_refine (algorithm (a)), fp64_b (algorithm (b))")
    ap.add_argument("--batch-count", type=int, default=512, help="c5_batch: number of problems")
    ap.add_argument("--batch-iters", type=int, default=3, help="c5_batch: refinement steps")
    ap.add_argument("--no-tune", action="store_true", help="c5_batch: no line-pass tuning")
    ap.add_argument("--batch-precision", default="fp32_refine", choices=("fp32_refine", "fp64", "fp32"),
                    help="c5_batch: precision mode of every problem")
    ap.add_argument("--heat-steps", type=int, default=10, help="heat: implicit Euler steps per timed step")
    ap.add_argument("--heat-precision", default="fp64", choices=("fp64", "fp32_refine", "fp32"))
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the timing of replays of one solve captured in a hipGraph")
    ap.add_argument("--tune", action="store_true", help="measure line-pass parameters first (N >= 2)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run one plain device copy of BYTES (profiler counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs one problem on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_1701_03967_amd import fftfem as fm
    fm.lib()
    if args.copy_calibration:
        copy_calibration(torch, args.copy_calibration)
    if args.workload == "transform1d":
        run_transform1d(args, torch, fm)
        return
    if args.workload == "heat":
        run_heat(args, torch, fm)
        return
    if args.workload == "long2d":
        run_long2d(args, torch, fm)
        return
    if args.workload == "c5_batch":
        run_batch(args, torch, fm)
        return

    def roofline_of(kt, prob, workload, steps_timed, mode=""):
        """Roofline of the dominant kernel of one mode (the most total time
        per step), from its mean HIP-event duration on the plan's stream."""
        if not kt:
            return None
        name, (avg_ms, cnt) = max(kt.items(), key=lambda kv: kv[1][0] * kv[1][1])
        by = kernel_bytes(name, prob.size, prob.N, prob.n)
        if by <= 0:
            return None
        gbs = by / (avg_ms * 1e-3) / 1e9
        ax = int(name.rsplit("_ax", 1)[1].rstrip("t")) if "_ax" in name else 0
        kname = profiler_kernel_name(name, prob.n, prob.N, prob.K[ax])
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": measured_traffic(workload, kname, mode),
                "kernel": name, "symbol": kname, "bytes_per_launch": by, "avg_ms": avg_ms,
                "launches_per_step": cnt / steps_timed}

    def run(name, full):
        w = inputs.WORKLOADS[name]
        prob = w.problem
        f_host = inputs.workload_rhs(name)
        f = torch.from_numpy(f_host).cuda()
        del f_host
        check = OracleCheck(torch, name, prob.shape)
        out = {"unknowns": prob.size}
        sols = {}
        for mode in args.modes.split(","):
            steps = args.steps if full else max(5, args.steps // 3)
            plan, u, ms, kt, st, extra = time_mode(fm, torch, prob, f, mode, steps, args.warmup, tune=args.tune,
                                                   graph=not args.no_graph)
            sols[mode] = u.clone()
            rec = {"ms": ms, "unknowns_per_s": prob.size / (ms * 1e-3), **extra}
            if mode == "fp32_refine":
                rec["iterations"] = st["iterations"]
                rec["rel_correction"] = st["rel_correction"]
            rec["converged"] = st["converged"]
            rec["stop"] = st["stop"]
            rec["err_vs_oracle"] = check(u)
            tol = 1e-5 if mode == "fp32" else 1e-10
            rec["err_tol"] = tol
            if rec["err_vs_oracle"] is not None:
                rec["err_ok"] = rec["err_vs_oracle"]["max"] <= tol
            rec["kernels_ms"] = {k: round(v[0], 5) for k, v in kt.items()}
            rec["kernels_per_step"] = {k: v[1] / min(steps, 10) for k, v in kt.items()}
            rec["stage_GBps"] = {k: round(kernel_bytes(k, prob.size, prob.N, prob.n) / (avg * 1e-3) / 1e9, 1)
                                 for k, (avg, _) in kt.items() if kernel_bytes(k, prob.size, prob.N, prob.n) > 0}
            # measured HBM bytes per launch of each kernel (committed counter
            # summaries; null when absent or taken on other sources)
            rec["stage_traffic_bytes"] = {
                k: measured_traffic(name, profiler_kernel_name(
                    k, prob.n, prob.N, prob.K[int(k.rsplit("_ax", 1)[1].rstrip("t")) if "_ax" in k else 0]), mode)
                for k in kt}
            step_bytes = sum(kernel_bytes(k, prob.size, prob.N, prob.n) * c / min(steps, 10) for k, (_, c) in kt.items())
            rec["bytes_per_step"] = step_bytes
            rec["step_GBps"] = round(step_bytes / (ms * 1e-3) / 1e9, 1)
            rec["roofline"] = roofline_of(kt, prob, name, min(steps, 10), mode)
            out[mode] = rec
            del plan
            print(f"[bench] {name} {mode}: {ms:.3f} ms/solve, err vs oracle {rec['err_vs_oracle']}",
                  file=sys.stderr, flush=True)
        if "fp64" in sols:
            ref = sols["fp64"]
            for mode, u in sols.items():
                if mode != "fp64":
                    out[mode]["rel_l2_vs_fp64"] = float(torch.linalg.norm(u - ref) / torch.linalg.norm(ref))
        del check
        return prob, out, sols

    prob, res, sols = run(args.workload, True)
    # headline: the faster of the two float64 solves (algorithms (a) and (b)
    # of Sect. 4 solve the same system to the same accuracy)
    f64 = [m for m in ("fp64", "fp64_b") if m in res]
    best_mode = min(f64, key=lambda m: res[m]["ms"]) if f64 else args.modes.split(",")[0]
    ms = res[best_mode]["ms"]
    value = prob.size / (ms * 1e-3)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": value / PAPER_UNKNOWNS_PER_S[args.workload] if args.workload in PAPER_UNKNOWNS_PER_S else None,
        "dtype": "f64" if best_mode.startswith("fp64") else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": prob.N, "n": prob.n, "K": list(prob.K),
                   "diff": list(prob.diff), "react": prob.react, "unknowns": prob.size,
                   "mode": best_mode, "algorithm": "b" if best_mode == "fp64_b" else "a", "rhs": inputs.WORKLOADS[args.workload].rhs,
                   "seed": inputs.WORKLOADS[args.workload].seed, "tuned": bool(args.tune)},
        "err_vs_oracle": res[best_mode]["err_vs_oracle"],
        "modes": {m: res[m] for m in res if m != "unknowns"},
        "roofline": res[best_mode]["roofline"],
    }
    if "fp64" in res and best_mode != "fp64":
        # algorithm (a), every axis transformed, beside the headline
        line["roofline_algorithm_a"] = res["fp64"]["roofline"]
    if args.also:
        del sols
        torch.cuda.empty_cache()
        p2, res2, sols2 = run(args.also, False)
        line["also"] = {args.also: {m: {k: v for k, v in res2[m].items() if k != "kernels_per_step"}
                                    for m in res2 if m != "unknowns"}}
        line["also"][args.also]["unknowns"] = p2.size
        del sols2
    if args.also and not args.no_batch:
        # the batched heat-step workload, 3 timed replays after 1 warm-up
        torch.cuda.empty_cache()
        ba = argparse.Namespace(**vars(args))
        ba.steps, ba.warmup, ba.quiet = 3, 1, True
        bl = run_batch(ba, torch, fm)
        line["also"]["c5_batch"] = {k: bl[k] for k in ("metric", "value", "unit", "ms_per_step", "dtype", "config",
                                                      "refinement", "roofline", "plan_s", "first_solve_s")}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, args.workload)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
