"""Pins of the channel-Fourier magnitude threshold in the oracle (reading F1):
the magnitudes are the orthonormal coordinates (Parseval), closed forms for
pure f = 0 and pure f = 1 content, zero threshold, and the c = 1 reduction
to Eq. 19."""
import numpy as np
import pytest

from oracle import filtering as f
from oracle import pipeline


def test_magnitudes_are_orthonormal_coordinates():
    S = np.random.default_rng(0).normal(size=(5, 4, 3, 8, 8))
    _, _, a = f.fourier_threshold(S, 0.0)
    energy = (S ** 2).sum(axis=-3)
    np.testing.assert_allclose(a[..., 0, :, :] ** 2 + a[..., 1, :, :] ** 2, energy, rtol=1e-12)
    np.testing.assert_array_equal(a[..., 1, :, :], a[..., 2, :, :])


def test_zero_threshold_keeps_everything():
    S = np.random.default_rng(1).normal(size=(3, 2, 3, 8, 8))
    St, keep, _ = f.fourier_threshold(S, 0.0)
    assert keep.all()
    np.testing.assert_allclose(St, S, atol=1e-12)


def test_pure_frequency_content():
    s = np.zeros((3, 8, 8))
    s[:, 2, 5] = 1.5                       # all channels equal: f = 0 only, a0 = sqrt(3) * 1.5
    St, keep, a = f.fourier_threshold(s, np.sqrt(3) * 1.5 - 1e-9)
    assert a[0, 2, 5] == pytest.approx(np.sqrt(3) * 1.5)
    assert a[1, 2, 5] == pytest.approx(0.0, abs=1e-12)
    np.testing.assert_allclose(St, s, atol=1e-12)
    St, _, _ = f.fourier_threshold(s, np.sqrt(3) * 1.5 + 1e-9)
    np.testing.assert_allclose(St, 0.0, atol=1e-12)
    r, phi = 2.0, 0.7                      # f = 1 only: a1 = r sqrt(3/2)
    t = np.zeros((3, 8, 8))
    t[:, 4, 1] = [r * np.cos(2 * np.pi * j / 3 + phi) for j in range(3)]
    St, keep, a = f.fourier_threshold(t, r * np.sqrt(1.5) - 1e-9)
    assert a[1, 4, 1] == pytest.approx(r * np.sqrt(1.5))
    assert keep[1, 4, 1] and keep[2, 4, 1] and not keep[0, 4, 1]
    np.testing.assert_allclose(St, t, atol=1e-12)
    St, _, _ = f.fourier_threshold(t, r * np.sqrt(1.5) + 1e-9)
    np.testing.assert_allclose(St, 0.0, atol=1e-12)


def test_gray_is_eq19():
    S = np.random.default_rng(2).normal(size=(4, 8, 1, 8, 8))
    a, ka, _ = f.fourier_threshold(S, 0.8)
    b, kb = f.hard_threshold(S, 0.8)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ka, kb)
    y = np.random.default_rng(3).normal(90.0, 20.0, size=(1, 30, 28))
    kw = dict(ps=8, stride=3, window=9, K=8)
    np.testing.assert_array_equal(pipeline.denoise(y, 20.0, fourier=True, **kw)["out"],
                                  pipeline.denoise(y, 20.0, **kw)["out"])


def test_rgb_variant_differs_but_stays_close():
    y = np.random.default_rng(4).normal(90.0, 20.0, size=(3, 30, 28))
    kw = dict(ps=8, stride=3, window=9, K=8)
    a = pipeline.denoise(y, 20.0, fourier=True, **kw)["out"]
    b = pipeline.denoise(y, 20.0, **kw)["out"]
    assert not np.allclose(a, b)
    assert np.abs(a - b).mean() < 5.0
