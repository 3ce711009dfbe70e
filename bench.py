#!/usr/bin/env python
"""Benchmark of the RAS-smoothed geometric multigrid for finite cell Stokes on one MI355X.

Workload (default): the 2D finite cell Stokes problem on a 512 x 512 background grid of the unit
square with 20 seeded non-overlapping disc obstacles (radii U[0.02, 0.06], alpha = 1e-8 inside),
parabolic inflow left, do-nothing outflow right, no-slip top/bottom, Q1-Q1 stabilised, 7-level
hierarchy, V(2,2) cycles with the restricted additive smoother (omega = 0.8) under the
cache_inverse policy, FP64. Synthetic inputs stand in for the paper's channel-flow grids.

A step is one V(2,2) cycle on the whole hierarchy (residuals, patch gathers, local solves,
restricted scatters, restriction, prolongation, coarsest solve). The headline value is the RAS
smoother throughput in fine-grid DoFs per second, counted as n_dof(finest) x (nu_pre + nu_post)
fine-grid sweeps per step, divided by the measured step time; it therefore includes every coarse-
level and transfer cost of the cycle. The same run also reports the fine-grid smoother alone, the
GMG solve time to a 1e-8 relative residual with p50/p99 latencies, the dominant kernel against the
HBM roofline, and the FP64 CPU oracle timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
Prints one JSON line on stdout; progress goes to stderr. Two helper modes for hardware counter runs
print a short JSON line instead: --cycles-only (the V-cycles alone, of the default workload or, with
--workload 3d_64 / 2d_4096, of a side workload) and --copy-calibration MIB (a plain device copy of known
size, the reference for scaling FETCH_SIZE / WRITE_SIZE to bytes).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector units, vendor figure


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(v, q):
    return float(np.percentile(np.asarray(v), q))


def algorithmic_bytes(kind: str, d: int, st: dict) -> float:
    """Bytes a kernel launch must move at minimum on one level (FP64 values, int32 indices).

    residual:          read x, b; write r; stored operator rows of the non-uniform nodes; one int
                       per node (operator code)
    residual_restrict: read x, b; write the coarse b; stored operator rows; one int per node
    apply_regular:     read r; one int per node; read+write x of the regular nodes; class rows
    apply_irregular:   the distinct stored row blocks (d+1)|S_i| of the streamed patches (wall
                       patches share theirs); read+write x and read r of those nodes; one int per
                       patch
    patch_solve:       read r; read+write x (local blocks are built on chip or, for cache_matrix,
                       read from the stored pattern values: added separately by the caller)
    sweep_fused:       read x, b; write the new x; distinct row blocks of the streamed patches;
                       distinct stored operator rows; two ints per node (patch class, operator code)
    """
    N = st["n_nodes"]
    nf = d + 1
    nsten = (2 * d + 2) * 3 ** d
    zs = d * 5 ** d + 3 ** d
    nreg = N - st["n_irregular"]
    rows = 8.0 * nsten * st["n_stencils"]
    if kind == "residual":
        return 8.0 * 3 * nf * N + rows + 4.0 * N
    if kind == "residual_restrict":
        nc = st["n_cells_axis"] // 2
        return 8.0 * 2 * nf * N + 8.0 * nf * (nc + 1) ** d + rows + 4.0 * N
    if kind == "apply_regular":
        return 8.0 * nf * N + 4.0 * N + 16.0 * nf * nreg + 8.0 * nf * zs * st["n_classes"]
    if kind == "apply_irregular":
        return 8.0 * nf * st["irregular_cols"] + 24.0 * nf * st["n_irregular"] + 4.0 * st["n_irregular"]
    if kind == "patch_solve":
        return 8.0 * 3 * nf * N
    if kind == "sweep_fused":
        return sweep_minimum_bytes(d, st) + 8.0 * N
    if kind in ("restrict", "prolong"):
        return 8.0 * nf * N * 1.25 if d == 2 else 8.0 * nf * N * 1.125
    return 0.0


def band_cholesky_flops(n: int, bw: int) -> int:
    """Floating-point operations of a right-looking Cholesky of an n x n matrix of half bandwidth bw,
    counting every add, multiply, divide and square root once: per column, the square root, the
    divisions of the m = min(bw, n - 1 - k) entries below the diagonal and the multiply-subtract
    updates of the m (m + 1) / 2 entries of the trailing lower triangle."""
    total = 0
    for k in range(n):
        m = min(bw, n - 1 - k)
        total += 1 + m + m * (m + 1)
    return total


def patch_solve_flops(d: int) -> int:
    """Operations of one local solve y = L_i^-1 g_i of the cache_matrix and cache_none policies
    (Eq. 15), as the patch kernel runs it: L_i = [[I_d (x) K, B], [B^T, C]] with K the 5^d velocity
    block of half bandwidth 5^(d-1) + ... + 1 in lexicographic order, B the 3^d pressure columns of each
    velocity component.
    * banded Cholesky K = L L^T;
    * forward substitution L V = [B_c | g_c | e_centre] for every component c (3^d + 2 columns);
    * Schur complement S = C - sum_c V_c^T V_c and the reduced right-hand side;
    * dense Cholesky of -S and the two triangular solves for the pressures;
    * the d velocity rows of the centre node.
    Assembling L_i (cache_none) comes on top and is not counted."""
    nv, npr = 5 ** d, 3 ** d
    bw = sum(5 ** k for k in range(d))
    mc = (nv - 1) // 2
    ncol = npr + 2
    chol_k = band_cholesky_flops(nv, bw)
    fwd_col = sum(2 * (i - max(0, i - bw)) + 1 for i in range(nv))
    schur = npr * npr * (2 * d * nv + 1) + d * npr * 2 * (nv - mc) + npr * (2 * d * nv + 1) + d * 2 * (nv - mc)
    chol_s = npr * npr + band_cholesky_flops(npr, npr - 1)
    tri = sum(2 * i + 2 for i in range(npr)) + sum(2 * (npr - 1 - i) + 2 for i in range(npr))
    centre = d * 2 * npr
    return chol_k + d * ncol * fwd_col + schur + chol_s + tri + centre


# Cut-cell element data of the byte model: K (symmetric, 10 / 36 distinct doubles) and the d blocks
# B_c (32 / 192 doubles) per cut cell, 2D / 3D.
CUT_CELL_DOUBLES = {2: 42, 3: 228}


def sweep_bytes(d: int, st: dict) -> float:
    """Algorithmic bytes of one fused cache_inverse sweep on a level (FP64): read x and b and write the
    new x, 3 n_DoF values; the (d+1) |S_i| inverse-row values of every distinct streamed row block;
    the element data of every cut cell (CUT_CELL_DOUBLES). Shared class rows and reference data are
    level constants and count nothing."""
    nf = d + 1
    return 8.0 * (3 * nf * st["n_nodes"] + nf * st["irregular_cols"] + CUT_CELL_DOUBLES[d] * st["n_cut_cells"])


def sweep_minimum_bytes(d: int, st: dict) -> float:
    """Fused minimum of one cache_inverse sweep: read x, b, write x, the distinct row blocks of the
    streamed patches and the distinct stored operator rows, each once (FP64)."""
    nf = d + 1
    nsten = (2 * d + 2) * 3 ** d
    return 8.0 * (3 * nf * st["n_nodes"] + nf * st["irregular_cols"] + nsten * st["n_stencils"])


def time_vcycles(torch, h, x, b, steps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        h.vcycle(x, b)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def time_sweeps(torch, h, x, b, count):
    """Per-sweep latency (ms) of `count` smoother calls of two sweeps each, halved: the V-cycle
    smooths in pairs (2D cache_inverse: one fused launch per sweep, ping-pong buffers)."""
    lat = []
    for _ in range(count):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        h.smooth(x, b, 2)
        e1.record()
        lat.append((e0, e1))
    torch.cuda.synchronize()
    return [a.elapsed_time(z) / 2 for a, z in lat]


def time_solves(torch, h, b, count, rtol=1e-8, max_iter=200):
    ms, its, rels = [], [], []
    for _ in range(count):
        x = h.zeros()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _, it, rel, _, rc = h.solve(b, x=x, rtol=rtol, max_iter=max_iter)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
        its.append(it)
        rels.append(rel)
    return ms, its, rels


def dominant_kernel(torch, h, x, b, steps, d):
    """Profile `steps` V-cycles with the library's event timers (on the launch stream) and return
    the kernel kind/level with the largest total time, with its average launch time."""
    h.profile(True)
    h.profile_reset()
    for _ in range(steps):
        h.vcycle(x, b)
    torch.cuda.synchronize()
    prof = h.profile_read()
    h.profile(False)
    (kind, lev), (tot, cnt) = max(prof.items(), key=lambda kv: kv[1][0])
    total_all = sum(v[0] for v in prof.values())
    avg_ms = tot / cnt
    timing = "per-launch events of the library profiler"
    if kind == "sweep_fused" and lev == h.fine:
        # the fine-level fused sweep alone: 50 smoother calls of two fused launches each between one
        # pair of events on the launch stream (no per-launch events in the timed region)
        h.smooth(x, b, 2)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(50):
            h.smooth(x, b, 2)
        e1.record()
        torch.cuda.synchronize()
        avg_ms = e0.elapsed_time(e1) / 100
        timing = "100 back-to-back launches between two events"
    st = h.stats(lev)
    model = algorithmic_bytes(kind, d, st)
    nbytes = sweep_bytes(d, st) if kind == "sweep_fused" else model
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    table = {f"{k}@L{l}": {"avg_us": round(v[0] / v[1] * 1e3, 3), "launches": v[1],
                           "share": round(v[0] / total_all, 4)} for (k, l), v in sorted(prof.items())}
    return {
        "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(f"{kind}@L{lev}"),
        "kernel": f"{kind}@L{lev}", "avg_launch_us": round(avg_ms * 1e3, 3), "avg_launch_timing": timing,
        "algorithmic_bytes_per_launch": int(nbytes),
        "bytes_model": "8 [3 n_DoF + (d+1) sum_irr |S_i| + e_d n_cut], e_d = 42 (2D) / 228 (3D)"
                       if kind == "sweep_fused" else "per-kernel minimum (algorithmic_bytes)",
        "builder_model_bytes_per_launch": int(model), "time_share": round(tot / total_all, 4),
    }, table


def kernel_sources_sha256() -> str:
    """Hash over the HIP/C++ sources of the library: counter figures taken on other sources are stale."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_11636_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if not fn.endswith((".hip", ".cpp", ".h", ".inl")):
            continue
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel_key: str):
    """HBM bytes per launch of `kernel_key` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    (profiles/hbm_traffic.json, scaled by a plain-copy calibration), or None when no figure exists
    for it or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256") != kernel_sources_sha256():
        return None
    return int(rec["traffic_bytes"])


def cpu_baseline(prob, budget_s=10.0, budget_1core_s=5.0):
    """The FP64 oracle (as it stands) on the host cores: cache_inverse-form V(2,2) cycles on the same
    problem, repeated until about `budget_s` seconds of cycles have run, on all cores and then on one
    core (about `budget_1core_s` seconds, at least two cycles). The oracle's inverse-row set-up runs
    first, untimed."""
    from oracle.oracle import MODE_INVERSE, Oracle, max_threads, set_threads
    t0 = time.perf_counter()
    o = Oracle(prob)
    b = o.rhs()
    x = o.vcycle(np.zeros_like(b), b, mode=MODE_INVERSE)  # builds the inverse rows on every level
    setup_s = time.perf_counter() - t0
    steps = 0
    t0 = time.perf_counter()
    while steps < 2 or time.perf_counter() - t0 < budget_s:
        x = o.vcycle(x, b, mode=MODE_INVERSE)
        steps += 1
    dt = (time.perf_counter() - t0) / steps
    cores = max_threads()
    set_threads(1)
    try:
        steps1 = 0
        t0 = time.perf_counter()
        while steps1 < 2 or time.perf_counter() - t0 < budget_1core_s:
            x = o.vcycle(x, b, mode=MODE_INVERSE)
            steps1 += 1
        dt1 = (time.perf_counter() - t0) / steps1
    finally:
        set_threads(cores)
    nd = o.ndofs(o.fine)
    work = nd * (prob.nu_pre + prob.nu_post)
    return {
        "value": round(work / dt, 1), "unit": "DOF/s", "cores": cores, "kind": "oracle",
        "value_1core": round(work / dt1, 1),
        "sample": f"{prob.name}: {steps} V({prob.nu_pre},{prob.nu_post}) cycles of the FP64 oracle in "
                  f"cache_inverse form on {cores} threads after its untimed {setup_s:.1f} s inverse-row set-up, "
                  f"{dt * 1e3:.1f} ms per cycle; then {steps1} cycles on one thread, {dt1 * 1e3:.1f} ms per cycle",
    }


def policy_extras(torch, fcgmg, prob, sweeps=4, integrated=False):
    """The factorising policies on `prob`; with `integrated`, cache_none also with every block
    assembled from the window's element integrals, its cut cells integrated during the sweep."""
    out = {}
    runs = [(fcgmg.CACHE_MATRIX, False), (fcgmg.CACHE_NONE, False)] + ([(fcgmg.CACHE_NONE, True)] if integrated else [])
    for pol, integ in runs:
        t0 = time.perf_counter()
        h = fcgmg.Hierarchy(prob, pol)
        if integ:
            h.set_cache_none_assembly(True)
        setup = time.perf_counter() - t0
        b = h.rhs()
        x = h.zeros()
        h.smooth(x, b, 1)
        lat = time_sweeps(torch, h, x, b, sweeps)
        ms = float(np.median(lat))
        vc_ms, _ = time_vcycles(torch, h, x, b, 2)  # every level under this policy
        st = h.stats()
        # one local solve per node and sweep, FP64 vector arithmetic: the fraction of the FP64 peak
        flops = patch_solve_flops(prob.dim) * st["n_nodes"]
        tflops = flops / (ms * 1e-3) / 1e12
        name = fcgmg.POLICY_NAMES[pol] + ("_integrated" if integ else "")
        out[name] = {
            "sweep_ms_p50": round(ms, 4), "vcycle_ms": round(vc_ms, 3),
            "smoother_dof_per_s": round(h.ndofs() / (ms * 1e-3), 1),
            "cached_bytes_finest": st["cached_bytes"], "device_bytes": h.device_bytes(),
            "setup_s": round(setup, 3), "solve_gflop_per_sweep": round(flops / 1e9, 3),
            "achieved_tflops": round(tflops, 4), "fp64_vector_peak_frac": round(tflops / FP64_VECTOR_PEAK_TFLOPS, 5)}
        h.close()
        log(f"  {name}: sweep {ms:.3f} ms")
    return out


def immersed_extra(torch, fcgmg, prob, solves=5):
    """The same workload with the obstacle surfaces as no-slip Dirichlet boundaries (immersed
    Nitsche, cache_inverse): set-up, the V-cycle, and the time to 1e-8 of the standalone GMG and of
    FGMRES(30) preconditioned by one V-cycle; then one sweep under each policy that takes these
    terms (2D: all three, 3D: cache_inverse)."""
    import dataclasses
    p = dataclasses.replace(prob, immersed_nitsche=1)
    out = {"workload": prob.name + "_immersed_nitsche"}
    pol = {}
    for solver, tag in ((fcgmg.SOLVER_GMG, "gmg"), (fcgmg.SOLVER_FGMRES, "fgmres")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = fcgmg.Hierarchy(p, fcgmg.CACHE_INVERSE, solver=solver)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        b = h.rhs()
        rec = {"setup_s": round(setup_s, 3)}
        if solver == fcgmg.SOLVER_GMG:
            xx = h.zeros()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            h.vcycle(xx, b)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(10):
                h.vcycle(xx, b)
            e1.record()
            torch.cuda.synchronize()
            rec["cycle_us"] = round(e0.elapsed_time(e1) / 10 * 1e3, 1)
        try:
            h.solve(b, rtol=1e-8, max_iter=300)
            ms, its, rels = time_solves(torch, h, b, solves, max_iter=300)
            rec.update({"converged": True, "solve_ms_p50": round(pct(ms, 50), 3), "cycles": int(np.median(its)),
                        "rel_res": float(np.max(rels))})
        except fcgmg.FcgmgError as e:
            rec.update({"converged": False, "error": str(e)[:160]})
        out[tag] = rec
        if solver == fcgmg.SOLVER_GMG:
            # the cache_inverse sweep on this hierarchy (the policy comparison below)
            x = h.zeros()
            lat = time_sweeps(torch, h, x, b, 3)
            pol["cache_inverse"] = {"sweep_ms_p50": round(float(np.median(lat)), 4), "device_bytes": h.device_bytes()}
        h.close()
    # the other policies of Sec. 3.1.2 with these terms (2D: dense LU of the local blocks at every
    # application for cache_matrix and cache_none; 3D takes cache_inverse only)
    policies = ((fcgmg.CACHE_MATRIX, "cache_matrix"), (fcgmg.CACHE_NONE, "cache_none"))
    for policy, name in () if p.dim == 3 else policies:
        h = fcgmg.Hierarchy(p, policy)
        b = h.rhs()
        x = h.zeros()
        lat = time_sweeps(torch, h, x, b, 3)
        pol[name] = {"sweep_ms_p50": round(float(np.median(lat)), 4), "device_bytes": h.device_bytes()}
        h.close()
    out["policies"] = pol
    return out


def precision_extra(torch, fcgmg, prob, solves=5):
    """Time to 1e-8 on one workload for the standalone FP64 GMG, the mixed-precision GMG (FP32 V-cycles
    inside FP64 iterative refinement) and FGMRES(30) preconditioned by one FP64 or FP32 V-cycle:
    cycles, the cycle alone, and the distance of each iterate from the FP64 GMG one."""
    out = {"workload": prob.name}
    xs = {}
    for prec, solver, tag in ((fcgmg.PREC_FP64, fcgmg.SOLVER_GMG, "fp64"), (fcgmg.PREC_MIXED, fcgmg.SOLVER_GMG, "mixed"),
                              (fcgmg.PREC_FP64, fcgmg.SOLVER_FGMRES, "fgmres_fp64"),
                              (fcgmg.PREC_MIXED, fcgmg.SOLVER_FGMRES, "fgmres_mixed")):
        h = fcgmg.Hierarchy(prob, fcgmg.CACHE_INVERSE, precision=prec, solver=solver)
        b = h.rhs()
        h.solve(b, rtol=1e-8, max_iter=200)
        ms, its, rels = time_solves(torch, h, b, solves)
        x, _, _, _, _ = h.solve(b, rtol=1e-8, max_iter=200)
        xs[tag] = x.cpu().numpy()
        if solver == fcgmg.SOLVER_FGMRES:
            out[tag] = {"solve_ms_p50": round(pct(ms, 50), 3), "solve_ms_p99": round(pct(ms, 99), 3),
                        "cycles": int(np.median(its)), "rel_res": float(np.max(rels)), "device_bytes": h.device_bytes()}
            h.close()
            continue
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        if prec == fcgmg.PREC_MIXED:
            e = h.zeros()
            h.vcycle_fp32(b, out=e)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(10):
                h.vcycle_fp32(b, out=e)
            e1.record()
        else:
            xx = h.zeros()
            e0.record()
            for _ in range(10):
                h.vcycle(xx, b)
            e1.record()
        torch.cuda.synchronize()
        out[tag] = {"solve_ms_p50": round(pct(ms, 50), 3), "solve_ms_p99": round(pct(ms, 99), 3),
                    "cycles": int(np.median(its)), "rel_res": float(np.max(rels)),
                    "cycle_us": round(e0.elapsed_time(e1) / 10 * 1e3, 1), "device_bytes": h.device_bytes()}
        h.close()
    for tag in ("mixed", "fgmres_fp64", "fgmres_mixed"):
        out[tag]["rel_diff_vs_fp64_gmg"] = float(np.linalg.norm(xs[tag] - xs["fp64"]) / np.linalg.norm(xs["fp64"]))
        out[tag]["speedup_vs_fp64_gmg"] = round(out["fp64"]["solve_ms_p50"] / out[tag]["solve_ms_p50"], 3)
    return out


def serving_extra(fcgmg, inputs, n_req=200, rate=200.0, workers=4, seed=0, n_warm=60, rate_warm=10.0):
    """Solve server under a Poisson arrival stream: requests drawn uniformly from a pool of seeded
    obstacle problems (2D 128^2..1024^2 with 20 discs, 3D 32^3..96^3 with 40 spheres; alpha 1e-8;
    FP64 or mixed precision per problem), FGMRES(30) preconditioned by the V-cycle, tolerance 1e-8.
    Cold start: every hierarchy is set up by its first request. Latency is submit to completion.
    The stream of `rate` requests per second exceeds what one GPU serves, so its latencies measure
    the backlog; a second stream of `n_warm` requests at `rate_warm` per second, on the same server
    with its hierarchies resident, measures the latency below capacity."""
    rng = np.random.default_rng(seed)
    pool = []
    for n, lv in ((128, 5), (256, 6), (512, 7), (1024, 8)):
        for sd in (0, 1):
            pool.append((inputs.config2(sd, n_cells=n, n_levels=lv), fcgmg.PREC_MIXED if sd else fcgmg.PREC_FP64))
    for n, lv in ((32, 4), (48, 4), (64, 5), (96, 5)):
        pool.append((inputs.config3(0, n_cells=n, n_levels=lv), fcgmg.PREC_MIXED))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    picks = rng.integers(0, len(pool), n_req)
    srv = fcgmg.Server(workers=workers)
    t0 = time.perf_counter()
    ids = []
    for k in range(n_req):
        delay = t0 + arrivals[k] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        p, prec = pool[picks[k]]
        ids.append(srv.submit(p, precision=prec, solver=fcgmg.SOLVER_FGMRES))
    res = [srv.wait(i)[1] for i in ids]
    wall = time.perf_counter() - t0
    resident, n_res = srv.resident()
    arrivals2 = np.cumsum(rng.exponential(1.0 / rate_warm, n_warm))
    picks2 = rng.integers(0, len(pool), n_warm)
    t1 = time.perf_counter()
    ids2 = []
    for k in range(n_warm):
        delay = t1 + arrivals2[k] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        p, prec = pool[picks2[k]]
        ids2.append(srv.submit(p, precision=prec, solver=fcgmg.SOLVER_FGMRES))
    res2 = [srv.wait(i)[1] for i in ids2]
    wall2 = time.perf_counter() - t1
    srv.close()
    ok2 = [r for r in res2 if r["status"] == fcgmg.OK]
    lat2 = [r["t_total_ms"] for r in ok2]
    solve2 = [r["t_solve_ms"] for r in ok2]
    ok = [r for r in res if r["status"] == fcgmg.OK]
    lat = [r["t_total_ms"] for r in ok]
    solve = [r["t_solve_ms"] for r in ok]
    return {
        "requests": n_req, "arrival_rate_per_s": rate, "workers": workers, "pool": len(pool),
        "completed": len(ok), "throughput_req_per_s": round(len(ok) / wall, 2),
        "latency_ms_p50": round(pct(lat, 50), 2), "latency_ms_p99": round(pct(lat, 99), 2),
        "solve_ms_p50": round(pct(solve, 50), 2), "solve_ms_p99": round(pct(solve, 99), 2),
        "setup_ms_total": round(float(sum(r["t_setup_ms"] for r in ok)), 1),
        "cache_hits": int(sum(r["cache_hit"] for r in ok)),
        "max_rel_res": float(max(r["rel_res"] for r in ok)),
        "policies": {fcgmg.POLICY_NAMES[k]: int(sum(r["policy"] == k for r in ok)) for k in (0, 1, 2)},
        "resident_bytes_end": resident, "resident_hierarchies_end": n_res, "wall_s": round(wall, 2),
        "below_capacity": {
            "requests": n_warm, "arrival_rate_per_s": rate_warm, "completed": len(ok2),
            "throughput_req_per_s": round(len(ok2) / wall2, 2),
            "latency_ms_p50": round(pct(lat2, 50), 2) if ok2 else None,
            "latency_ms_p99": round(pct(lat2, 99), 2) if ok2 else None,
            "solve_ms_p50": round(pct(solve2, 50), 2) if ok2 else None,
            "solve_ms_p99": round(pct(solve2, 99), 2) if ok2 else None,
            "cache_hits": int(sum(r["cache_hit"] for r in ok2)), "wall_s": round(wall2, 2)},
    }


def fallback_plan(fcgmg, inputs, restart=30):
    """Pool and device-memory budget of serving_fallback_extra (host only): the budget is halfway
    between what the 512^2 problem needs under cache_none and under the faster of the other two
    policies (fcgmg_footprint_bytes of an FGMRES(`restart`) hierarchy plus the solution vector, as
    the server admits it). Returns (pool, budget, need(prob, policy))."""
    pool = [inputs.config2(0, n_cells=256, n_levels=6), inputs.config2(1, n_cells=256, n_levels=6), inputs.config2(0)]

    def need(prob, pol):
        ndof = (prob.dim + 1) * (prob.n_cells + 1) ** prob.dim
        return fcgmg.footprint_bytes(prob, pol, fcgmg.PREC_FP64, fcgmg.SOLVER_FGMRES, restart) + 8 * ndof

    big = pool[2]
    fast = min(need(big, fcgmg.CACHE_INVERSE), need(big, fcgmg.CACHE_MATRIX))
    budget = (need(big, fcgmg.CACHE_NONE) + fast) // 2
    assert need(big, fcgmg.CACHE_NONE) < budget < fast and need(pool[0], fcgmg.CACHE_INVERSE) < budget
    return pool, budget, need


def serving_fallback_extra(fcgmg, inputs, n_req=12, rate=8.0, workers=4, seed=2, restart=30):
    """Admission under memory pressure: FP64 FGMRES(`restart`) requests from 2D 256^2 (seeds 0, 1) and
    512^2 (seed 0) problems on a server whose device-memory budget lies between what the 512^2
    problem needs under cache_none and under the two faster policies, so that it is admitted with
    cache_none (Sec. 3.1.2's trade of speed for memory), while a 256^2 problem alone fits under
    cache_inverse. Cold start, Poisson arrivals; latency is submit to completion."""
    rng = np.random.default_rng(seed)
    pool, budget, need = fallback_plan(fcgmg, inputs, restart)
    big = pool[2]
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    picks = rng.integers(0, len(pool), n_req)
    srv = fcgmg.Server(workers=workers, hbm_budget=budget)
    t0 = time.perf_counter()
    ids = []
    for k in range(n_req):
        delay = t0 + arrivals[k] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(srv.submit(pool[picks[k]], solver=fcgmg.SOLVER_FGMRES, krylov_restart=restart))
    res = [srv.wait(i)[1] for i in ids]
    wall = time.perf_counter() - t0
    srv.close()
    ok = [r for r in res if r["status"] == fcgmg.OK]
    by_size = {}
    for k, r in zip(picks, res):
        if r["status"] != fcgmg.OK:
            continue
        key = f"{pool[k].n_cells}^2"
        d = by_size.setdefault(key, {fcgmg.POLICY_NAMES[q]: 0 for q in (0, 1, 2)})
        d[fcgmg.POLICY_NAMES[r["policy"]]] += 1
    lat = [r["t_total_ms"] for r in ok]
    return {
        "requests": n_req, "arrival_rate_per_s": rate, "workers": workers, "hbm_budget_bytes": int(budget),
        "need_bytes_512": {fcgmg.POLICY_NAMES[q]: int(need(big, q)) for q in (0, 1, 2)},
        "need_bytes_256_cache_inverse": int(need(pool[0], fcgmg.CACHE_INVERSE)),
        "completed": len(ok), "policies_by_size": by_size,
        "latency_ms_p50": round(pct(lat, 50), 2) if ok else None,
        "latency_ms_p99": round(pct(lat, 99), 2) if ok else None,
        "max_rel_res": float(max(r["rel_res"] for r in ok)) if ok else None,
        "wall_s": round(wall, 2),
    }


def serving_batched_extra(fcgmg, inputs, n_req=200, rate=200.0, workers=8, n_pool=32, seed=1):
    """Continuous batching: standalone GMG solves (V(2,2), FP64, cache_inverse, tolerance 1e-8) drawn
    from `n_pool` problems of the batching workload (2D, 64^2..256^2, 1..12 discs, alpha_f in
    {1e-6, 1e-8, 1e-10}), served with continuous batching on and off on the same request sequence,
    each from a cold start: a Poisson stream of `rate` requests per second, and the same requests
    submitted at once (a burst, which saturates the server). Latency is submit to completion."""
    out = {"requests": n_req, "workers": workers, "pool": n_pool,
           "poisson": serving_batched_run(fcgmg, inputs, n_req, rate, workers, n_pool, seed),
           "burst": serving_batched_run(fcgmg, inputs, n_req, None, workers, n_pool, seed)}
    out["poisson"]["arrival_rate_per_s"] = rate
    return out


def serving_batched_run(fcgmg, inputs, n_req, rate, workers, n_pool, seed):
    rng = np.random.default_rng(seed)
    pool = [inputs.batch_problem(k) for k in range(n_pool)]
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req)) if rate else np.zeros(n_req)
    picks = rng.integers(0, n_pool, n_req)
    out = {}
    for mode in (1, 0):
        srv = fcgmg.Server(workers=workers, continuous_batching=mode)
        t0 = time.perf_counter()
        ids = []
        for k in range(n_req):
            delay = t0 + arrivals[k] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            ids.append(srv.submit(pool[picks[k]], policy=fcgmg.CACHE_INVERSE))
        res = [srv.wait(i)[1] for i in ids]
        wall = time.perf_counter() - t0
        steps, cycles, max_batch = srv.stats()
        srv.close()
        ok = [r for r in res if r["status"] == fcgmg.OK]
        lat = [r["t_total_ms"] for r in ok]
        out["batching_on" if mode else "batching_off"] = {
            "completed": len(ok), "throughput_req_per_s": round(len(ok) / wall, 2),
            "latency_ms_p50": round(pct(lat, 50), 2), "latency_ms_p99": round(pct(lat, 99), 2),
            "cache_hits": int(sum(r["cache_hit"] for r in ok)), "max_rel_res": float(max(r["rel_res"] for r in ok)),
            "wall_s": round(wall, 2), "batched_steps": steps, "request_cycles": cycles,
            "mean_batch": round(cycles / steps, 2) if steps else None, "max_batch": max_batch}
    return out


def batch_extra(torch, fcgmg, inputs, n_prob=256, workers=4):
    """Batching workload: 256 independent 2D problems of uneven sizes (64^2..256^2, 1..12 discs,
    alpha_f in {1e-6, 1e-8, 1e-10}). Hierarchies are set up first (untimed). Measured: FGMRES(30)
    solves to 1e-8 one after another on one stream and through the solve server's concurrent
    workers; one V-cycle of all 256 problems one after another and as one batched cycle (one launch
    per cycle step, with one workgroup per tile or persistent sweeps); the batched standalone GMG
    solve (at most 60 cycles; the problems on which the standalone cycle does not converge are
    counted, not solved)."""
    probs = [inputs.batch_problem(k) for k in range(n_prob)]
    ndof = sum((p.dim + 1) * (p.n_cells + 1) ** p.dim for p in probs)
    # sequential: one stream, resident hierarchies
    hs = [fcgmg.Hierarchy(p, fcgmg.CACHE_INVERSE, solver=fcgmg.SOLVER_FGMRES) for p in probs]
    bs = [h.rhs() for h in hs]
    its = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h, b in zip(hs, bs):
        _, it, rel, _, rc = h.solve(b, rtol=1e-8, max_iter=200)
        its.append(it)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for h in hs:
        h.close()
    # batched: one launch per V-cycle step for all 256 problems (standalone GMG cycles)
    hs = [fcgmg.Hierarchy(p, fcgmg.CACHE_INVERSE) for p in probs]
    bs = [h.rhs() for h in hs]
    xs = [h.zeros() for h in hs]
    for h, x, b in zip(hs, xs, bs):
        h.vcycle(x, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        for h, x, b in zip(hs, xs, bs):
            h.vcycle(x, b)
    torch.cuda.synchronize()
    t_cyc_seq = (time.perf_counter() - t0) / 5
    bt = fcgmg.Batch(hs)
    bt.vcycle(xs, bs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        bt.vcycle(xs, bs)
    torch.cuda.synchronize()
    t_cyc_bat = (time.perf_counter() - t0) / 5
    # the same batched cycle with every fused sweep as one persistent launch
    bt.set_persistent(True)
    bt.vcycle(xs, bs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        bt.vcycle(xs, bs)
    torch.cuda.synchronize()
    t_cyc_per = (time.perf_counter() - t0) / 5
    bt.set_persistent(False)
    xs = [h.zeros() for h in hs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, bits, brel, brc = bt.solve(bs, xs=xs, rtol=1e-8, max_iter=60)
    torch.cuda.synchronize()
    t_bsolve = time.perf_counter() - t0
    bt.close()
    for h in hs:
        h.close()
    conv = [i for i, r in enumerate(brel) if r <= 1e-8]
    # server: warm pass sets the hierarchies up, the timed pass hits them
    srv = fcgmg.Server(workers=workers)
    for rid in [srv.submit(p, policy=fcgmg.CACHE_INVERSE, solver=fcgmg.SOLVER_FGMRES) for p in probs]:
        srv.wait(rid)
    t0 = time.perf_counter()
    res = [srv.wait(rid)[1] for rid in [srv.submit(p, policy=fcgmg.CACHE_INVERSE, solver=fcgmg.SOLVER_FGMRES)
                                         for p in probs]]
    t_srv = time.perf_counter() - t0
    srv.close()
    ok = sum(r["status"] == fcgmg.OK for r in res)
    return {
        "problems": n_prob, "total_dof": ndof, "sizes": sorted({p.n_cells for p in probs}),
        "cycles_median": int(np.median(its)), "cycles_max": int(max(its)),
        "sequential_s": round(t_seq, 3), "sequential_problems_per_s": round(n_prob / t_seq, 1),
        "server_workers": workers, "server_s": round(t_srv, 3), "server_problems_per_s": round(n_prob / t_srv, 1),
        "server_completed": ok, "server_cache_hits": int(sum(r["cache_hit"] for r in res)),
        "speedup": round(t_seq / t_srv, 3),
        "vcycle_all_sequential_ms": round(t_cyc_seq * 1e3, 3), "vcycle_all_batched_ms": round(t_cyc_bat * 1e3, 3),
        "vcycle_all_batched_persistent_ms": round(t_cyc_per * 1e3, 3),
        "batched_vcycle_dof_per_s": round(ndof * 4 / t_cyc_bat, 1),
        "batched_vcycle_speedup": round(t_cyc_seq / t_cyc_bat, 2),
        "batched_gmg_solve_s": round(t_bsolve, 3), "batched_gmg_converged": len(conv),
        "batched_gmg_cycles_median": int(np.median([bits[i] for i in conv])) if conv else None,
    }


def workload_extra(torch, fcgmg, prob, steps=20, warmup=3):
    t0 = time.perf_counter()
    h = fcgmg.Hierarchy(prob, fcgmg.CACHE_INVERSE)
    setup = time.perf_counter() - t0
    b = h.rhs()
    x = h.zeros()
    for _ in range(warmup):
        h.vcycle(x, b)
    ms, _ = time_vcycles(torch, h, x, b, steps)
    lat = time_sweeps(torch, h, x, b, 10)
    sw = float(np.median(lat))
    st = h.stats()
    nd = h.ndofs()
    fine = prob.n_levels - 1
    sbytes = sweep_bytes(prob.dim, st)
    if prob.dim == 2:
        keys = [f"sweep_fused@L{fine}"]
    else:
        keys = [f"residual@L{fine}", f"apply_regular@L{fine}", f"apply_irregular@L{fine}"]
    parts = [measured_traffic(k) for k in keys]
    roof = {"bound": "hbm", "kernels": keys, "algorithmic_bytes_per_sweep": int(sbytes),
            "sweep_us_p50": round(sw * 1e3, 2), "achieved": round(sbytes / (sw * 1e-3) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(sbytes / (sw * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": sum(parts) if all(p is not None for p in parts) else None}
    res = {
        "workload": prob.name, "n_dof": nd, "setup_s": round(setup, 3), "vcycle_ms": round(ms, 4),
        "value_dof_per_s": round(nd * (prob.nu_pre + prob.nu_post) / (ms * 1e-3), 1),
        "smoother_dof_per_s": round(nd / (sw * 1e-3), 1), "sweep_ms_p50": round(sw, 4),
        "sweep_min_bytes": int(sweep_minimum_bytes(prob.dim, st)),
        "sweep_gbs_vs_min_bytes": round(sweep_minimum_bytes(prob.dim, st) / (sw * 1e-3) / 1e9, 1),
        "n_irregular": st["n_irregular"], "n_cut_cells": st["n_cut_cells"], "device_bytes": h.device_bytes(),
        "roofline": roof,
    }
    h.close()
    return res


def autotune_extra(torch, fcgmg, prob, reps=20, steps=20):
    """Fused-sweep tile shapes: the V-cycle with the default shapes by level size, then the library's
    autotuner (every shape timed per level, the fastest kept) and the V-cycle again."""
    h = fcgmg.Hierarchy(prob, fcgmg.CACHE_INVERSE)
    b = h.rhs()
    x = h.zeros()
    for _ in range(3):
        h.vcycle(x, b)
    ms_default, _ = time_vcycles(torch, h, x, b, steps)
    t0 = time.perf_counter()
    res = h.autotune(reps=reps)
    tune_s = time.perf_counter() - t0
    for _ in range(3):
        h.vcycle(x, b)
    ms_tuned, _ = time_vcycles(torch, h, x, b, steps)
    shapes = [fcgmg.fused_shape(k) for k in range(fcgmg.N_FUSED_SHAPES)]
    levels = []
    for lev in range(1, h.n_levels):
        us = res["us"][lev]
        k = res["shape"][lev]
        levels.append({"level": lev, "n_cells": prob.level_cells(lev), "tuned": list(shapes[k]),
                       "us_per_shape": [round(u, 2) for u in us]})
    table = h.tuning_table(res)
    h.close()
    return {"workload": prob.name, "shapes_tile_x_tile_y_threads_waves_per_simd": [list(s) for s in shapes],
            "choice_by_level_cells": {k: list(v) for k, v in table.items()},
            "reps": reps, "tune_s": round(tune_s, 3), "vcycle_ms_default": round(ms_default, 4),
            "vcycle_ms_tuned": round(ms_tuned, 4), "levels": levels}


def stacked_extra(torch, fcgmg, prob, nrhs=8, reps=5):
    """Stacked right-hand sides on one geometry: two sweeps of nrhs vectors through fcgmg_smooth_multi
    (each streamed patch's rows read once per sweep for all vectors) against nrhs separate two-sweep
    smooth calls, per sweep of all vectors; then one V-cycle of every vector through fcgmg_vcycle_multi
    against nrhs fcgmg_vcycle calls."""
    h = fcgmg.Hierarchy(prob, fcgmg.CACHE_INVERSE)
    n = h.ndofs()
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    X = torch.randn(nrhs * n, dtype=torch.float64, device="cuda", generator=g)
    B = torch.randn(nrhs * n, dtype=torch.float64, device="cuda", generator=g)
    R = torch.zeros_like(X)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    h.smooth_multi(X, B, R, nrhs, 2)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        h.smooth_multi(X, B, R, nrhs, 2)
    e1.record()
    torch.cuda.synchronize()
    stacked = e0.elapsed_time(e1) / (2 * reps)
    xs = [X[k * n:(k + 1) * n] for k in range(nrhs)]
    bs = [B[k * n:(k + 1) * n] for k in range(nrhs)]
    e0.record()
    for _ in range(reps):
        for k in range(nrhs):
            h.smooth(xs[k], bs[k], 2)
    e1.record()
    torch.cuda.synchronize()
    separate = e0.elapsed_time(e1) / (2 * reps)
    # one V-cycle of every vector: fcgmg_vcycle_multi against nrhs fcgmg_vcycle calls
    h.vcycle_multi(X, B, nrhs)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        h.vcycle_multi(X, B, nrhs)
    e1.record()
    torch.cuda.synchronize()
    stacked_cycle = e0.elapsed_time(e1) / reps
    e0.record()
    for _ in range(reps):
        for k in range(nrhs):
            h.vcycle(xs[k], bs[k])
    e1.record()
    torch.cuda.synchronize()
    separate_cycle = e0.elapsed_time(e1) / reps
    h.close()
    return {"workload": prob.name, "nrhs": nrhs, "stacked_ms_per_sweep": round(stacked, 4),
            "separate_ms_per_sweep": round(separate, 4), "speedup": round(separate / stacked, 2),
            "stacked_dof_per_s": round(nrhs * n / (stacked * 1e-3), 1),
            "stacked_ms_per_vcycle": round(stacked_cycle, 4), "separate_ms_per_vcycle": round(separate_cycle, 4),
            "vcycle_speedup": round(separate_cycle / stacked_cycle, 2)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the policy / 3D / 4096^2 side measurements")
    ap.add_argument("--cycles-only", action="store_true",
                    help="run warmup + steps V-cycles of one workload and nothing else (for trace and counter runs)")
    ap.add_argument("--workload", choices=["2d_512", "3d_64", "2d_4096"], default="2d_512",
                    help="workload of --cycles-only: the bench workload (default), 3D 64^3 with 40 spheres, or "
                         "2D 4096^2 with 20 discs and 10 levels")
    ap.add_argument("--sweeps-only", action="store_true",
                    help="run warmup + steps single fine-level sweeps of --workload under --policy and nothing else "
                         "(for trace and counter runs of the factorising policies)")
    ap.add_argument("--policy", choices=["inverse", "matrix", "none", "none_integrated"], default="inverse",
                    help="cache policy of --sweeps-only")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run only a plain device-to-device copy of MIB MiB, 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sharded multi-GPU path is not implemented; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2403_11636_amd import fcgmg, inputs

    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "repeats": 5}), flush=True)
        return
    prob = inputs.config2(0)
    if (args.cycles_only or args.sweeps_only) and args.workload == "3d_64":
        prob = inputs.config3(0)
    elif (args.cycles_only or args.sweeps_only) and args.workload == "2d_4096":
        prob = inputs.config2(0, n_cells=4096, n_levels=10)
    if args.sweeps_only:
        pol = {"inverse": fcgmg.CACHE_INVERSE, "matrix": fcgmg.CACHE_MATRIX, "none": fcgmg.CACHE_NONE,
               "none_integrated": fcgmg.CACHE_NONE}[args.policy]
        h = fcgmg.Hierarchy(prob, pol)
        if args.policy == "none_integrated":
            h.set_cache_none_assembly(True)
        x, b = h.zeros(), h.rhs()
        for _ in range(args.warmup + args.steps):
            h.smooth(x, b, 1)
        torch.cuda.synchronize()
        print(json.dumps({"workload": prob.name, "policy": args.policy, "sweeps": args.warmup + args.steps,
                          "n_dof": h.ndofs()}), flush=True)
        h.close()
        return
    d = prob.dim
    log(f"setup {prob.name} (cache_inverse) ...")
    t0 = time.perf_counter()
    h = fcgmg.Hierarchy(prob, fcgmg.CACHE_INVERSE)
    setup_s = time.perf_counter() - t0
    nd = h.ndofs()
    b = h.rhs()
    x = h.zeros()
    for _ in range(args.warmup):
        h.vcycle(x, b)
    torch.cuda.synchronize()
    if args.cycles_only:
        for _ in range(args.steps):
            h.vcycle(x, b)
        torch.cuda.synchronize()
        print(json.dumps({"workload": prob.name, "vcycles": args.warmup + args.steps, "n_dof": nd}), flush=True)
        h.close()
        return
    log(f"timing {args.steps} V-cycles ...")
    ms_step, wall = time_vcycles(torch, h, x, b, args.steps)
    sweeps_per_step = prob.nu_pre + prob.nu_post
    value = nd * sweeps_per_step / (ms_step * 1e-3)

    log("fine-grid sweeps, solves, profile ...")
    lat = time_sweeps(torch, h, x, b, 100)
    sw50, sw99 = pct(lat, 50), pct(lat, 99)
    solve_ms, its, rels = time_solves(torch, h, b, 20)
    roof, table = dominant_kernel(torch, h, x, b, max(5, args.steps // 5), d)
    st = h.stats()
    sweep_min = sweep_minimum_bytes(d, st)

    out = {
        "metric": "RAS smoother DOF/s, GMG solve time to 1e-8 rel. residual; p50/p99 latency",
        "value": round(value, 1),
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "2D finite cell Stokes, 512x512 background grid, 20 seeded discs r~U[0.02,0.06], "
                        "alpha=1e-8, Q1-Q1 stabilised, inflow/do-nothing, 7-level GMG V(2,2), RAS smoother "
                        "cache_inverse, omega=0.8",
            "n_dof_finest": nd, "levels": prob.n_levels, "step": "one V(2,2) cycle",
            "value_definition": "n_dof(finest) x 4 fine-grid sweeps per cycle / cycle time",
            "parallelism": "1 GPU",
        },
        "smoother": {
            "sweep_us_p50": round(sw50 * 1e3, 2), "sweep_us_p99": round(sw99 * 1e3, 2),
            "fine_sweep_dof_per_s": round(nd / (sw50 * 1e-3), 1),
            "sweep_min_bytes": int(sweep_min),
            "sweep_gbs_vs_min_bytes": round(sweep_min / (sw50 * 1e-3) / 1e9, 1),
        },
        "solve": {
            "rtol": 1e-8, "iterations": int(np.median(its)), "rel_res": float(np.max(rels)),
            "ms_p50": round(pct(solve_ms, 50), 3), "ms_p99": round(pct(solve_ms, 99), 3), "count": len(solve_ms),
            "setup_s": round(setup_s, 3),
        },
        "roofline": roof,
        "kernels": table,
        "wall_s_timed_region": round(wall, 4),
    }
    h.close()
    if not args.no_extras:
        log("policies ...")
        out["policies"] = policy_extras(torch, fcgmg, prob, integrated=True)
        out["policies"]["cache_inverse"] = {"sweep_ms_p50": round(sw50, 4),
                                           "smoother_dof_per_s": round(nd / (sw50 * 1e-3), 1),
                                           "cached_bytes_finest": st["cached_bytes"]}
        log("3D 64^3 ...")
        out["extra_3d"] = workload_extra(torch, fcgmg, inputs.config3(0))
        log("3D 64^3 policies ...")
        out["policies_3d"] = policy_extras(torch, fcgmg, inputs.config3(0), sweeps=3)
        out["roofline_3d"] = out["extra_3d"]["roofline"]
        log("precision: FP64 vs mixed ...")
        out["precision"] = [precision_extra(torch, fcgmg, inputs.config2(0)), precision_extra(torch, fcgmg, inputs.config3(0))]
        log("stacked right-hand sides ...")
        out["stacked_rhs"] = [stacked_extra(torch, fcgmg, inputs.config3(0)), stacked_extra(torch, fcgmg, inputs.config2(0))]
        log("immersed Nitsche ...")
        out["immersed"] = immersed_extra(torch, fcgmg, inputs.config2(0))
        log("immersed Nitsche, 3D ...")
        out["immersed_3d"] = immersed_extra(torch, fcgmg, inputs.config3(0))
        log("batching ...")
        out["batching"] = batch_extra(torch, fcgmg, inputs)
        log("serving ...")
        out["serving"] = serving_extra(fcgmg, inputs)
        log("serving under a memory budget (policy fallback) ...")
        out["serving_fallback"] = serving_fallback_extra(fcgmg, inputs)
        log("serving with continuous batching ...")
        out["serving_batched"] = serving_batched_extra(fcgmg, inputs)
        log("2D 4096^2 ...")
        big = inputs.config2(0, n_cells=4096, n_levels=10)
        big.name = "2d_20discs_4096_seed0"
        out["extra_2d_4096"] = workload_extra(torch, fcgmg, big)
        out["roofline_4096"] = out["extra_2d_4096"]["roofline"]
        log("fused-sweep shape autotuning ...")
        out["autotune"] = [autotune_extra(torch, fcgmg, prob), autotune_extra(torch, fcgmg, big, reps=10)]
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(prob)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
