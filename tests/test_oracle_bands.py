"""Pins of the general band count (HSI tubes, reading H1) in the oracle: the
band-mean guide against a direct rounding of the exact rational mean, the
reduction to the grey pipeline when every band is the same image, the basis
invariants for other c (unitary Fourier slices, real tensors, eigenvalue
sums), and perfect reconstruction at tau = 0."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import basis, matching, pipeline


def _round_half_even(fr: Fraction) -> int:
    fl = fr.numerator // fr.denominator
    rem = fr - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        return fl + 1
    return fl


@pytest.mark.parametrize("c", [2, 4, 5, 7, 31])
def test_band_mean_is_the_rounded_rational_mean(c):
    rng = np.random.default_rng(c)
    q = rng.integers(-(1 << 20) + 1, 1 << 20, size=(c, 6, 7))
    q[:, 0, 0] = 3                       # exact ties: sum = 3c -> 3
    q[:, 0, 1] = np.arange(c) - c // 2   # symmetric sums around zero
    if c % 2 == 0:
        q[:, 0, 2] = 0
        q[0, 0, 2] = c // 2              # mean 1/2 -> 0 (even)
        q[:, 0, 3] = 0
        q[0, 0, 3] = -(c // 2) * 3       # mean -3/2 -> -2 (even)
    g = matching.band_mean(q)
    for y in range(6):
        for x in range(7):
            want = _round_half_even(Fraction(int(q[:, y, x].sum()), c))
            assert int(g[y, x]) == want
    assert np.abs(g).max() < (1 << 20)


@pytest.mark.parametrize("c", [2, 5])
def test_equal_bands_reduce_to_grey(c):
    y1 = np.random.default_rng(11).normal(100.0, 20.0, size=(1, 26, 24))
    yc = np.repeat(y1, c, axis=0)
    kw = dict(ps=8, stride=3, window=9, K=8)
    r1 = pipeline.denoise(y1, 20.0, **kw)
    rc = pipeline.denoise(yc, 20.0, **kw)
    np.testing.assert_array_equal(rc["idx"], r1["idx"])
    for ch in range(c):
        np.testing.assert_allclose(rc["out"][ch], r1["out"][0], atol=1e-9)


@pytest.mark.parametrize("c", [2, 4, 6, 7])
def test_basis_invariants_for_other_band_counts(c):
    y = np.random.default_rng(20 + c).normal(80.0, 30.0, size=(c, 20, 21))
    UF, VF, U, V, eU, eV = basis.global_basis(y, 8, 3)
    for F in (UF, VF):
        for f in range(c):
            np.testing.assert_allclose(F[f].conj().T @ F[f], np.eye(8), atol=1e-12)
    np.testing.assert_allclose(np.fft.ifft(UF, axis=0).imag, 0.0, atol=1e-14)
    P = basis.ref_patches(y, 8, 3)
    Ph = np.fft.fft(P, axis=1)
    for f in range(c // 2 + 1):
        e = float((np.abs(Ph[:, f]) ** 2).sum())
        assert eU[f].sum() == pytest.approx(e, rel=1e-12)
        assert eV[f].sum() == pytest.approx(e, rel=1e-12)
    if c % 2 == 0:                        # f = c/2 is a real eigenproblem
        np.testing.assert_allclose(UF[c // 2].imag, 0.0, atol=1e-12)


@pytest.mark.parametrize("c", [2, 5])
def test_zero_threshold_reconstructs_other_band_counts(c):
    y = np.random.default_rng(30 + c).normal(90.0, 25.0, size=(c, 22, 20))
    r = pipeline.denoise(y, 0.0, ps=8, stride=3, window=9, K=8)
    np.testing.assert_allclose(r["out"], y, atol=1e-9)
