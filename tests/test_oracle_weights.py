"""Pins of the weighted aggregation reading (Eq. 2 with w_g = 1/max(1, kept
coefficients of group g)) in the oracle: a hand-computed pixel, the
reduction to uniform weights, the weight rule, and convexity."""
import numpy as np
import pytest

from oracle import filtering as f
from oracle import pipeline


def test_hand_computed_pixel():
    # two groups of one 1x1-channel patch each, both covering pixel (0, 0)
    # of a 9x9 image; group 0 estimate 10 with weight 1/4, group 1 estimate 40
    # with weight 1/2: x = (10/4 + 40/2) / (1/4 + 1/2) = 30
    est = np.zeros((2, 1, 1, 8, 8))
    est[0, 0, 0] = 10.0
    est[1, 0, 0] = 40.0
    idx = np.array([[0], [0]])
    num, cnt = f.aggregate(est, idx, 1, 9, 9, 8, np.array([0.25, 0.5]))
    assert num[0, 0, 0] / cnt[0, 0] == pytest.approx(30.0)
    assert cnt[0, 0] == pytest.approx(0.75)
    assert cnt[8, 8] == 0.0


def test_weight_rule():
    keep = np.zeros((3, 2, 1, 8, 8), dtype=bool)
    keep[0, 0, 0, 0, :5] = True
    keep[1] = True
    w = f.group_weights(keep)
    np.testing.assert_allclose(w, [1 / 5, 1 / 128, 1.0])


def test_constant_weights_reduce_to_uniform():
    rng = np.random.default_rng(1)
    est = rng.normal(size=(6, 4, 3, 8, 8))
    idx = rng.integers(0, 9, size=(6, 4)) * 17 + rng.integers(0, 9, size=(6, 4))
    n0, c0 = f.aggregate(est, idx, 3, 17, 17, 8)
    n1, c1 = f.aggregate(est, idx, 3, 17, 17, 8, np.full(6, 0.3))
    m = c0 > 0
    np.testing.assert_allclose((n1 / c1[None])[:, m], (n0 / c0[None])[:, m], rtol=1e-12)


def test_zero_threshold_keeps_everything_and_equals_uniform():
    y = np.random.default_rng(2).normal(100.0, 20.0, size=(3, 28, 26))
    kw = dict(ps=8, stride=3, window=9, K=8)
    a = pipeline.denoise(y, 0.0, **kw)["out"]
    b = pipeline.denoise(y, 0.0, weighted=True, **kw)["out"]
    np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-9)


def test_weighted_output_is_a_convex_combination():
    y = np.random.default_rng(3).normal(100.0, 25.0, size=(1, 30, 30))
    r = pipeline.denoise(y, 25.0, ps=8, stride=3, window=9, K=8, weighted=True)
    u = pipeline.denoise(y, 25.0, ps=8, stride=3, window=9, K=8)
    assert np.isfinite(r["out"]).all()
    # same groups and estimates, other weights: the outputs differ but stay
    # within the range of the estimates (bounded by the uniform output's
    # neighbourhood of the data range)
    assert not np.allclose(r["out"], u["out"])
    assert r["out"].min() >= y.min() - 5 * 25 and r["out"].max() <= y.max() + 5 * 25
    c = np.full((3, 24, 24), 42.5)
    rc = pipeline.denoise(c, 10.0, ps=8, stride=3, window=9, K=8, weighted=True)["out"]
    np.testing.assert_allclose(rc, 42.5, rtol=1e-12)
