"""Pins of the A-Haar-tSVD noise-level adjustment in the oracle (Sec. III.D,
Eq. 21-22): brute-force eigenvalues of the explicitly built circulant, the
closed form of Eq. 21, constructed groups with known ranks, the vote rule and
the sub-image composition."""
import numpy as np
import pytest

from oracle import adaptive, pipeline


def circ_matrix(G):
    """circ(G) built entry by entry: column j stacks p_{i-j} (mod K), i = 0..K-1."""
    K, d = G.shape
    M = np.zeros((K * d, K))
    for j in range(K):
        for i in range(K):
            M[i * d:(i + 1) * d, j] = G[(i - j) % K]
    return M


@pytest.mark.parametrize("K,d,seed", [(2, 3, 0), (4, 5, 1), (8, 6, 2), (16, 4, 3)])
def test_eigenvalues_match_brute_force(K, d, seed):
    G = np.random.default_rng(seed).normal(size=(K, d))
    M = circ_matrix(G)
    brute = np.sort(np.linalg.eigvalsh(M.T @ M))
    # circ(G) circ(G)^T has the same nonzero spectrum
    big = np.sort(np.linalg.eigvalsh(M @ M.T))[-K:]
    lam = np.sort(adaptive.circulant_eigenvalues(G))
    np.testing.assert_allclose(lam, brute, rtol=1e-10, atol=1e-9)
    np.testing.assert_allclose(lam, big, rtol=1e-9, atol=1e-8)


@pytest.mark.parametrize("K", [4, 8, 32])
def test_eq21_closed_form_and_eigenvector(K):
    G = np.random.default_rng(K).normal(size=(K, 3, 8, 8))
    lam = adaptive.circulant_eigenvalues(G)
    sgn = np.array([(-1.0) ** (i + 1) for i in range(K)])     # (-1)^i, i = 1..K
    alt = (sgn[:, None] * G.reshape(K, -1)).sum(axis=0)
    assert lam[K // 2] == pytest.approx(float(alt @ alt), rel=1e-12)
    # u-hat = (-1, 1, ..., -1, 1)/sqrt(K) is an eigenvector of circ(G)^T circ(G)
    M = circ_matrix(G.reshape(K, -1))
    u = sgn / np.sqrt(K)
    np.testing.assert_allclose(M.T @ M @ u, lam[K // 2] * u, rtol=1e-10, atol=1e-8)


def test_rank_of_constructed_groups():
    K = 32
    q = np.random.default_rng(5).normal(size=(3, 8, 8))
    same = np.stack([q] * K)                        # no difference between patches
    assert adaptive.rank_position(adaptive.circulant_eigenvalues(same)) == 1
    alt = np.stack([q * (-1.0) ** i for i in range(K)])   # all energy in the alternating mode
    assert adaptive.rank_position(adaptive.circulant_eigenvalues(alt)) == K
    # a hand-made spectrum: lambda_{K/2} = 5 with three smaller values
    lams = np.full(8, 9.0)
    lams[[1, 2, 7]] = [1.0, 2.0, 4.0]
    lams[4] = 5.0
    assert adaptive.rank_position(lams) == 4
    lams[3] = 5.0                                  # an equal value is not below
    assert adaptive.rank_position(lams) == 4


def test_vote_rule():
    assert adaptive.adjust_sigma([3, 5, 20], 24.0, 1.2, 13) == pytest.approx(20.0)
    assert adaptive.adjust_sigma([3, 20, 20], 24.0, 1.2, 13) == 24.0
    assert adaptive.adjust_sigma([13, 14], 24.0, 1.2, 13) == 24.0      # tie keeps sigma_est
    assert adaptive.adjust_sigma([13, 13, 14, 2], 12.0, 1.5, 13) == pytest.approx(8.0)


def test_group_ranks_use_slot_order():
    """The ranks come from the groups of the match (gather in slot order)."""
    rng = np.random.default_rng(7)
    y = rng.normal(100.0, 20.0, size=(3, 24, 24))
    idx = np.stack([rng.choice(17 * 17, size=8, replace=False) for _ in range(5)])
    idx = (idx // 17) * 24 + idx % 17
    r = adaptive.group_ranks(y, idx, [4, 0, 2])
    from oracle.filtering import gather_groups
    G = gather_groups(y, idx[[4, 0, 2]], 8)
    expect = [1 + int((adaptive.circulant_eigenvalues(g) < adaptive.circulant_eigenvalues(g)[4]).sum())
              for g in G]
    assert list(r) == expect


def test_sub_images_are_independent_images():
    rng = np.random.default_rng(11)
    y = rng.normal(120.0, 25.0, size=(1, 40, 48))
    subs = [(0, 0, 40, 24), (0, 24, 40, 24)]
    kw = dict(ps=8, stride=3, window=9, K=8)
    samples = [np.array([0, 5, 9]), np.array([1, 2, 3])]
    out, sig, rk = adaptive.a_haar_tsvd(y, 25.0, subs, samples, **kw)
    for (y0, x0, h, w), s in zip(subs, sig):
        ref = pipeline.denoise(y[:, y0:y0 + h, x0:x0 + w], s, **kw)["out"]
        np.testing.assert_array_equal(out[:, y0:y0 + h, x0:x0 + w], ref)
    for s, r in zip(sig, rk):
        assert s == adaptive.adjust_sigma(r, 25.0)
