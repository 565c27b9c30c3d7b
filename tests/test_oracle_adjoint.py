"""Pins for the oracle's adjoint of the frozen denoiser (derived from
Eq. 18-20 and Eq. 2 with the grouping, masks and basis held fixed)."""
import numpy as np
import pytest

from oracle import adjoint, pipeline
from paper_2508_10307_amd import synth


def _frozen(C, seed, H=26, W=30, K=8):
    y = synth.tiny(seed, C, H, W)
    r = pipeline.denoise(y, 20.0, 8, 3, 9, K, return_mask=True)
    return y, r, K


@pytest.mark.parametrize("C", [1, 3])
def test_dot_product_identity(C):
    y, r, K = _frozen(C, 80 + C)
    rng = np.random.default_rng(C)
    a = rng.normal(size=y.shape)
    z = rng.normal(size=y.shape)
    Da, cnt = adjoint.frozen_forward(a, r["idx"], r["mask"], r["U"], r["V"], K)
    Dtz = adjoint.frozen_adjoint(z, r["idx"], r["mask"], r["U"], r["V"], cnt, K)
    lhs, rhs = np.vdot(Da, z), np.vdot(a, Dtz)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("C", [1, 3])
def test_frozen_forward_equals_pipeline(C):
    y, r, K = _frozen(C, 90 + C)
    x, cnt = adjoint.frozen_forward(y, r["idx"], r["mask"], r["U"], r["V"], K)
    np.testing.assert_allclose(x, r["out"], atol=1e-10)
    np.testing.assert_array_equal(cnt, r["cnt"])


def test_gradient_matches_central_fd_of_frozen_loss():
    y, r, K = _frozen(3, 95)
    clean = synth.clean_image(95, 0, 3, 26, 30, 4)
    args = (r["idx"], r["mask"], r["U"], r["V"])
    n = y.size

    def loss(v):
        x, _ = adjoint.frozen_forward(v, *args, K)
        return np.sum((x - clean) ** 2) / n
    x, cnt = adjoint.frozen_forward(y, *args, K)
    g = adjoint.mse_loss_grad(x, clean, *args, cnt, K, n)
    rng = np.random.default_rng(3)
    h = 1e-3
    for _ in range(6):
        p = tuple(rng.integers(0, s) for s in y.shape)
        e = np.zeros(y.shape)
        e[p] = h
        fd = (loss(y + e) - loss(y - e)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-7 * max(1.0, abs(g[p]))


def test_gradient_matches_unfrozen_fd_away_from_kinks():
    # With the basis held fixed, re-running matching and thresholding at
    # y +- h e_p gives the same loss derivative as the frozen adjoint whenever
    # neither the groups nor the masks change (probes that move them are skipped).
    y, r, K = _frozen(1, 96)
    clean = synth.clean_image(96, 0, 1, 26, 30, 4)
    n = y.size
    U, V = r["U"], r["V"]
    x, cnt = adjoint.frozen_forward(y, r["idx"], r["mask"], U, V, K)
    g = adjoint.mse_loss_grad(x, clean, r["idx"], r["mask"], U, V, cnt, K, n)
    rng = np.random.default_rng(4)
    h, checked = 1e-3, 0
    for _ in range(40):
        p = tuple(rng.integers(0, s) for s in y.shape)
        e = np.zeros(y.shape, dtype=np.float64)
        e[p] = h
        runs = [pipeline.denoise(y + sgn * e, 20.0, 8, 3, 9, K, U=U, V=V, return_mask=True)
                for sgn in (1, -1)]
        if any((not np.array_equal(q["idx"], r["idx"])) or
               (not np.array_equal(q["mask"], r["mask"])) for q in runs):
            continue
        lp, lm = (np.sum((q["out"] - clean) ** 2) / n for q in runs)
        assert abs((lp - lm) / (2 * h) - g[p]) <= 1e-7 * max(1.0, abs(g[p]))
        checked += 1
        if checked == 5:
            break
    assert checked >= 3


def test_threshold_multiplier_gradient_is_zero_away_from_kinks():
    # tau enters only through the frozen mask: if no |S| lies within h*sigma
    # of tau, moving lambda by +-h changes nothing.
    y = synth.tiny(97, 3, 16, 16)
    sigma, h = 20.0, 1e-4
    r = pipeline.denoise(y, sigma, 8, 3, 9, 4)
    S = np.abs(pipeline.group_coefficients(y, r["idx"], r["U"], r["V"], 4))
    lams = np.linspace(2.5, 2.9, 401)
    gaps = [np.abs(S - l * sigma).min() for l in lams]
    lam = float(lams[int(np.argmax(gaps))])
    assert max(gaps) > h * sigma
    a = pipeline.denoise(y, sigma, 8, 3, 9, 4, tau_mult=lam + h)["out"]
    b = pipeline.denoise(y, sigma, 8, 3, 9, 4, tau_mult=lam - h)["out"]
    assert np.array_equal(a, b)
