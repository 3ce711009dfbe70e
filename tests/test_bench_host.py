"""Host logic of bench.py (no GPU): argument handling, the byte model and the traffic figure's tie to
the kernel sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    p = run_bench("--gpus", "2")
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_unknown_workload_is_refused():
    p = run_bench("--cycles-only", "--workload", "4d_8")
    assert p.returncode == 2
    assert "--workload" in p.stderr


STATS = {"n_nodes": 263169, "n_irregular": 22000, "irregular_cols": 1250000, "n_stencils": 15000,
         "n_classes": 2, "n_cells_axis": 512, "n_cut_cells": 3295}


@pytest.mark.parametrize("d", [2, 3])
def test_sweep_bytes_follow_the_byte_model(d):
    # 8 [3 n_DoF + (d+1) sum_irr |S_i| + e_d n_cut], e_d = 42 (2D) / 228 (3D)
    nf = d + 1
    e_d = 42 if d == 2 else 228
    expect = 8.0 * (3 * nf * STATS["n_nodes"] + nf * STATS["irregular_cols"] + e_d * STATS["n_cut_cells"])
    assert bench.sweep_bytes(d, STATS) == expect
    for key in ("n_nodes", "irregular_cols", "n_cut_cells"):
        st = dict(STATS)
        st[key] += 1
        assert bench.sweep_bytes(d, st) > bench.sweep_bytes(d, STATS)


@pytest.mark.parametrize("d", [2, 3])
def test_fused_sweep_bytes_are_the_minimum_plus_the_class_codes(d):
    # the fused sweep moves the unfused minimum and one more int per node for each of two tables
    # (patch class, operator code): 8 bytes per node
    assert bench.algorithmic_bytes("sweep_fused", d, STATS) - bench.sweep_minimum_bytes(d, STATS) == 8.0 * STATS["n_nodes"]


def test_sweep_minimum_grows_with_each_term():
    base = bench.sweep_minimum_bytes(2, STATS)
    for key in ("n_nodes", "irregular_cols", "n_stencils"):
        st = dict(STATS)
        st[key] += 1
        assert bench.sweep_minimum_bytes(2, st) > base
    # x read, b read, x written: 3 (d+1) doubles per node
    st = dict(STATS, irregular_cols=0, n_stencils=0)
    assert bench.sweep_minimum_bytes(2, st) == 8.0 * 3 * 3 * STATS["n_nodes"]


def test_unknown_kernel_kind_has_no_byte_model():
    assert bench.algorithmic_bytes("no_such_kernel", 2, STATS) == 0.0


def test_measured_traffic_follows_the_kernel_sources(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as f:
        rec = json.load(f)["sweep_fused@L6"]
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: rec["source_sha256"])
    assert bench.measured_traffic("sweep_fused@L6") == int(rec["traffic_bytes"])
    assert bench.measured_traffic("no_such_kernel@L0") is None
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "0" * 64)
    assert bench.measured_traffic("sweep_fused@L6") is None


@pytest.mark.parametrize("n", [1, 2, 9, 25])
def test_band_cholesky_count_reduces_to_dense_and_diagonal(n):
    # full band: sum over the columns of 1 + 2m + m^2, m = n-1-k (the dense Cholesky count)
    assert bench.band_cholesky_flops(n, n - 1) == n + n * (n - 1) + (n - 1) * n * (2 * n - 1) // 6
    # no band: one square root per diagonal entry
    assert bench.band_cholesky_flops(n, 0) == n


def test_patch_solve_count_is_below_dense_lu_and_grows_with_dimension():
    for d in (2, 3):
        size = d * 5 ** d + 3 ** d  # 59 / 402 DoFs of a patch
        assert 0 < bench.patch_solve_flops(d) < 2 * size ** 3 // 3
    assert bench.patch_solve_flops(3) > 50 * bench.patch_solve_flops(2)


def test_fallback_leg_budget_forces_cache_none_for_the_large_problem():
    # The serving leg under memory pressure: with nothing else resident, the 512^2 problem fits its
    # budget only under cache_none, while a 256^2 problem fits under cache_inverse (footprints are
    # host-only planning, no GPU).
    from paper_2403_11636_amd import fcgmg, inputs
    pool, budget, need = bench.fallback_plan(fcgmg, inputs)
    big = pool[2]
    assert big.n_cells == 512
    assert need(big, fcgmg.CACHE_NONE) <= budget
    assert need(big, fcgmg.CACHE_INVERSE) > budget and need(big, fcgmg.CACHE_MATRIX) > budget
    for small in pool[:2]:
        assert small.n_cells == 256 and need(small, fcgmg.CACHE_INVERSE) <= budget
