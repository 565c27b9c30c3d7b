"""Host check of the Haar arrangement the filters use (CPU, no GPU).

The filters run the group-mode Haar transform (Eq. 9) as unnormalised
butterflies (u + v, u - v) in two lane layouts: the vector-ALU filter does
the levels inside a lane (SPL slots per lane) and then across lanes; the
MFMA filter pairs slots 2b, 2b+1 across lanes and then does the block levels
in registers.  The unnormalised forward transform is D H (D = diag 2^(l/2),
l the level of the coefficient left in slot k), so a coefficient is compared
with tau 2^(l/2), and each kept coefficient is weighted by 2^-l before the
unscaled inverse butterflies (which apply H^T D).  This simulates both
layouts in FP64 and checks the thresholded reconstruction, and the keep
decisions, against the oracle's orthonormal H_K.
"""
import numpy as np
import pytest

from oracle.haar import haar_matrix


def ctz(x):
    return (x & -x).bit_length() - 1


def level(k, K):
    return ctz(K) if k == 0 else ctz(k) + 1


def haar_row(k, K):
    if k == 0:
        return 0
    L = ctz(k) + 1
    return (K >> L) + (k >> L)


def threshold(coef, K, tau):
    keep = np.array([abs(coef[k]) >= tau * 2 ** (level(k, K) / 2) for k in range(K)])
    w = np.array([2.0 ** -level(k, K) for k in range(K)])
    return np.where(keep, coef * w, 0.0), keep


def cross(col, NL, m):
    new = col.copy()
    for kl in range(NL):
        if kl & (m - 1) == 0:
            o = col[kl ^ m]
            new[kl] = (o - col[kl]) if (kl & m) else (col[kl] + o)
    return new


def valu_layout(x, K, SPL, tau):
    NL = K // SPL
    X = x.reshape(NL, SPL).copy()
    st = 1
    while st < SPL:
        for j in range(0, SPL, 2 * st):
            u, v = X[:, j].copy(), X[:, j + st].copy()
            X[:, j], X[:, j + st] = u + v, u - v
        st *= 2
    m = 1
    while m < NL:
        X[:, 0] = cross(X[:, 0], NL, m)
        m *= 2
    c, keep = threshold(X.reshape(-1), K, tau)
    X = c.reshape(NL, SPL)
    m = NL // 2
    while m >= 1:
        X[:, 0] = cross(X[:, 0], NL, m)
        m //= 2
    st = SPL // 2
    while st >= 1:
        for j in range(0, SPL, 2 * st):
            u, v = X[:, j].copy(), X[:, j + st].copy()
            X[:, j], X[:, j + st] = u + v, u - v
        st //= 2
    return X.reshape(-1), keep


def mfma_layout(x, K, tau):
    NB = K // 2
    S = x.reshape(NB, 2).copy()
    a0, a1 = S[:, 0].copy(), S[:, 1].copy()
    S[:, 0], S[:, 1] = a0 + a1, a0 - a1
    w = 1
    while w < NB:
        for b in range(0, NB, 2 * w):
            u, v = S[b, 0], S[b + w, 0]
            S[b, 0], S[b + w, 0] = u + v, u - v
        w *= 2
    c, keep = threshold(S.reshape(-1), K, tau)
    S = c.reshape(NB, 2)
    w = NB // 2
    while w >= 1:
        for b in range(0, NB, 2 * w):
            u, v = S[b, 0], S[b + w, 0]
            S[b, 0], S[b + w, 0] = u + v, u - v
        w //= 2
    a0, a1 = S[:, 0].copy(), S[:, 1].copy()
    S[:, 0], S[:, 1] = a0 + a1, a0 - a1
    return S.reshape(-1), keep


def reference(x, K, tau):
    H = haar_matrix(K)
    c = H @ x
    keep_rows = np.abs(c) >= tau
    return H.T @ np.where(keep_rows, c, 0.0), np.array([keep_rows[haar_row(k, K)] for k in range(K)])


@pytest.mark.parametrize("K,SPL", [(2, 1), (4, 1), (8, 1), (16, 2), (32, 4), (64, 8)])
def test_valu_layout_matches_orthonormal_haar(K, SPL):
    rng = np.random.default_rng(K)
    for _ in range(40):
        x = rng.normal(0, 10, K)
        tau = abs(rng.normal(0, 8))
        y, keep = valu_layout(x, K, SPL, tau)
        ref, keep_ref = reference(x, K, tau)
        np.testing.assert_array_equal(keep, keep_ref)
        np.testing.assert_allclose(y, ref, atol=1e-9)


@pytest.mark.parametrize("K", [4, 8, 16, 32])
def test_mfma_layout_matches_orthonormal_haar(K):
    rng = np.random.default_rng(100 + K)
    for _ in range(40):
        x = rng.normal(0, 10, K)
        tau = abs(rng.normal(0, 8))
        y, keep = mfma_layout(x, K, tau)
        ref, keep_ref = reference(x, K, tau)
        np.testing.assert_array_equal(keep, keep_ref)
        np.testing.assert_allclose(y, ref, atol=1e-9)


def test_plain_inverse_without_weights_is_wrong():
    # the weights are needed: without them the unscaled inverse of the
    # pyramid is not a multiple of the identity
    K, SPL = 8, 1
    x = np.arange(1.0, K + 1)
    NL = K
    X = x.reshape(NL, SPL).copy()
    m = 1
    while m < NL:
        X[:, 0] = cross(X[:, 0], NL, m)
        m *= 2
    m = NL // 2
    while m >= 1:
        X[:, 0] = cross(X[:, 0], NL, m)
        m //= 2
    y = X.reshape(-1)
    assert not np.allclose(y / y[0] * x[0], x)
