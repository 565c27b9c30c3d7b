"""Host logic of bench.py (no GPU): the multi-GPU refusal, the work models
behind the roofline entries, the kernel names it reports and the stored
counter figures' source check."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_direct_filter_flops_per_group():
    # c = 3, K = 32: 32 * 2 * 11776 + 4 * 32 * 3 * 64 + 2 * 32 * 3 * 64
    assert bench.filter_flops_per_group(3, 32) == 790528
    assert bench.filter_flops_per_group(1, 16) == 16 * 2 * 2048 + 6 * 16 * 64


def test_window_candidates_by_enumeration():
    # separable per-axis count against a direct enumeration of every
    # reference's truncated window (the reference itself excluded)
    H, W, s, w = 40, 33, 3, 11
    r = (w - 1) // 2
    ys, xs = bench.ref_positions(H - 7, s), bench.ref_positions(W - 7, s)
    total = 0
    for y in ys:
        for x in xs:
            ny = min(H - 8, y + r) - max(0, y - r) + 1
            nx = min(W - 8, x + r) - max(0, x - r) + 1
            total += ny * nx - 1
    assert bench.window_candidates(H, W, s, w) == (total, len(ys) * len(xs))


def test_reported_kernel_names():
    # the instantiations the library launches for the benchmarked workloads
    assert bench.match_kernel_name(3, 3, 31, 0, 3) == "void hts::k_match<0, 3, 1, 2, 1>(hts::Launch)"
    assert bench.match_kernel_name(3, 2, 39, 0, 3) == "void hts::k_match<0, 3, 1, 2, 0>(hts::Launch)"
    assert bench.match_kernel_name(3, 3, 31, 1, 3) == "void hts::k_match<1, 1, 1, 2, 1>(hts::Launch)"
    assert bench.match_kernel_name(1, 3, 31, 0, 1) == "void hts::k_match<0, 1, 1, 1, 1>(hts::Launch)"
    assert bench.filter_kernel_name(3, 32, True, True) == "void hts::k_filter<3, 4, 0, 0, 1, 0, 0>(hts::Launch)"


def test_shortlist_summary_percentiles():
    h = np.zeros(130, np.int64)
    h[31] = 50
    h[32] = 30
    h[40] = 20
    h[129] = 3
    out = bench.shortlist_summary(h, 32)
    assert out["references"] == 103 and out["overflow"] == 3
    assert out["median"] == 31 and out["p90"] == 40 and out["max"] == 40
    assert out["below_k_minus_1"] == 0 and out["k_minus_1"] == 31


def test_stored_counter_figures_follow_the_sources():
    k = next(iter(bench.PROFILED))
    sha, figs = bench.PROFILED[k]
    tune = next(iter(figs))
    key = next(iter(figs[tune]))
    expect = figs[tune][key] if sha == bench.sources_sha() else None
    assert bench.profiled(k, key, tune) == expect
    assert bench.profiled("no such kernel", key, tune) is None
    assert bench.profiled(k, key, -1) is None or sha != bench.sources_sha()
