"""Pins of the threshold-gradient surrogate (reading S1) in the oracle: the
analytic dL/dtau equals central finite differences of the relaxed forward
map (grouping, basis and coverage frozen), and the relaxed map tends to the
hard one as the width shrinks."""
import numpy as np
import pytest

from oracle import adjoint, pipeline


@pytest.mark.parametrize("C,K", [(1, 8), (3, 4)])
def test_tau_gradient_matches_finite_differences(C, K):
    rng = np.random.default_rng(10 + C)
    y = rng.normal(100.0, 20.0, size=(C, 26, 24))
    r = pipeline.denoise(y, 20.0, ps=8, stride=3, window=9, K=K)
    idx, U, V, cnt = r["idx"], r["U"], r["V"], r["cnt"]
    g = rng.normal(size=y.shape)
    tau, eps = 2.7 * 20.0, 2.0
    ana = adjoint.tau_gradient(y, g, idx, U, V, cnt, K, tau, eps)
    h = 1e-3
    lp = float((g * adjoint.soft_forward(y, idx, U, V, K, tau + h, eps, cnt)).sum())
    lm = float((g * adjoint.soft_forward(y, idx, U, V, K, tau - h, eps, cnt)).sum())
    fd = (lp - lm) / (2 * h)
    assert ana == pytest.approx(fd, rel=1e-5, abs=1e-9)
    assert abs(ana) > 0


def test_soft_map_tends_to_the_hard_one():
    rng = np.random.default_rng(20)
    y = rng.normal(100.0, 20.0, size=(1, 26, 24))
    r = pipeline.denoise(y, 20.0, ps=8, stride=3, window=9, K=8)
    xs = adjoint.soft_forward(y, r["idx"], r["U"], r["V"], 8, 54.0, 1e-4, r["cnt"])
    np.testing.assert_allclose(xs, r["out"], atol=1e-3)
