"""Pins for the oracle's Haar matrix (Sec. II.D Eq. 8-9) and the circulant
eigen-facts that motivate it (Sec. III.B.2 Eq. 13-16, Sec. III.D Eq. 21)."""
import os

import numpy as np
import pytest

from oracle.haar import haar_matrix


def _read_golden(path):
    mats, cur, name = {}, None, None
    r = 1.0 / np.sqrt(2.0)
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line[0].isalpha():
            name, cur = line, []
            mats[name] = cur
            continue
        row = []
        for tok in line.split():
            if tok.endswith("*r"):
                row.append(float(tok[:-2]) * r)
            else:
                row.append(float(tok))
        cur.append(row)
    return {k: np.array(v) for k, v in mats.items()}


def test_printed_h2_and_worked_h4(golden_dir):
    g = _read_golden(os.path.join(golden_dir, "haar_h2_h4.txt"))
    np.testing.assert_allclose(haar_matrix(2), g["H2"], atol=1e-15)
    np.testing.assert_allclose(haar_matrix(4), g["H4"], atol=1e-15)


@pytest.mark.parametrize("K", [2, 4, 8, 16, 32, 64])
def test_orthogonal_and_dc_row(K):
    H = haar_matrix(K)
    np.testing.assert_allclose(H @ H.T, np.eye(K), atol=1e-14)
    np.testing.assert_allclose(H[0], np.full(K, 1.0 / np.sqrt(K)), atol=1e-15)


@pytest.mark.parametrize("K", [8, 16])
def test_haar_rows_are_piecewise_constant_differences(K):
    # Every row after the first sums to zero (a difference of two adjacent
    # dyadic blocks) and takes at most two distinct non-zero magnitudes of
    # opposite sign on a contiguous support.
    H = haar_matrix(K)
    for row in H[1:]:
        assert abs(row.sum()) < 1e-14
        nz = np.nonzero(np.abs(row) > 1e-14)[0]
        assert nz[-1] - nz[0] + 1 == len(nz)
        half = len(nz) // 2
        assert np.all(row[nz[:half]] > 0) and np.all(row[nz[half:]] < 0)


def test_non_power_of_two_rejected():
    for K in (0, 1, 3, 6, 12):
        with pytest.raises(ValueError):
            haar_matrix(K)


def _circ_group(p):
    """circ(G) of Eq. 13: row i holds p_{i}, p_{i-1}, ..., cyclically."""
    K = len(p)
    return np.vstack([np.concatenate([p[(i - j) % K] for j in range(K)]) for i in range(K)])


@pytest.mark.parametrize("K", [4, 8, 16])
def test_eq16_dominant_eigenpair_is_haar_dc_row(K):
    rng = np.random.default_rng(K)
    p = [rng.uniform(0, 255, 3 * 4) for _ in range(K)]      # non-negative patches
    M = _circ_group(p)
    A = M @ M.T
    rsum = np.sum(p, axis=0)
    u = np.full(K, 1.0 / np.sqrt(K))
    np.testing.assert_allclose(A @ u, (rsum @ rsum) * u, rtol=1e-12)
    w = np.linalg.eigvalsh(A)
    assert abs(w[-1] - rsum @ rsum) <= 1e-9 * w[-1]
    np.testing.assert_allclose(haar_matrix(K)[0], u, atol=1e-15)


@pytest.mark.parametrize("K", [4, 8, 32])
def test_eq21_alternating_eigenpair(K):
    rng = np.random.default_rng(100 + K)
    p = [rng.normal(size=5) for _ in range(K)]
    A = _circ_group(p) @ _circ_group(p).T
    s = sum(((-1) ** (i + 1)) * p[i] for i in range(K))
    u = np.array([(-1) ** (i + 1) for i in range(K)], dtype=float) / np.sqrt(K)
    np.testing.assert_allclose(A @ u, (s @ s) * u, rtol=1e-10, atol=1e-10)
