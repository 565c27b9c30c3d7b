"""Pins for the oracle's grouping (Sec. III.A Eq. 10, Alg. 1 Step 1).

The brute-force matcher below is written independently of oracle.matching:
pure Python integers, explicit loops over every candidate and pixel, its own
rounding and its own top-K selection by repeated minimum extraction.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import matching
from oracle.grid import ref_grid, ref_positions, window
from paper_2508_10307_amd import synth


def _q(v):
    """Round 256*v half to even with Python's exact Fraction arithmetic."""
    x = Fraction(float(v)) * 256
    fl = x.numerator // x.denominator
    rem = x - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return max(-(2 ** 20 - 1), min(2 ** 20 - 1, fl))


def brute_match(y, ps, stride, w, K, num=6, den=5):
    C, H, W = y.shape
    q = [[[_q(y[c, i, j]) for j in range(W)] for i in range(H)] for c in range(C)]
    Hp, Wp = H - ps + 1, W - ps + 1
    r = (w - 1) // 2

    def axis_refs(n):
        out, v = [], 0
        while v < n:
            out.append(v)
            v += stride
        if out[-1] != n - 1:
            out.append(n - 1)
        return out

    def guide(c_sel, i, j):
        if C == 1:
            return q[0][i][j]
        if c_sel == "G":
            return q[1][i][j]
        return q[0][i][j] + q[1][i][j] + q[2][i][j]

    rows = []
    for ry in axis_refs(Hp):
        for rx in axis_refs(Wp):
            sel = "G"
            if C == 3:
                n2 = [sum(q[c][ry + a][rx + b] ** 2 for a in range(ps) for b in range(ps))
                      for c in range(3)]
                # ||G|| >= max(||R||, ||B||)/gamma  <=>  (num/den)^2 nG >= max(nR, nB)
                sel = "G" if Fraction(num, den) ** 2 * n2[1] >= max(n2[0], n2[2]) else "S"
            cands = []
            for cy in range(max(0, ry - r), min(Hp - 1, ry + r) + 1):
                for cx in range(max(0, rx - r), min(Wp - 1, rx + r) + 1):
                    if (cy, cx) == (ry, rx):
                        continue
                    d = 0
                    for a in range(ps):
                        for b in range(ps):
                            e = guide(sel, ry + a, rx + b) - guide(sel, cy + a, cx + b)
                            d += e * e
                    cands.append((d, cy * W + cx))
            chosen = []
            for _ in range(K - 1):
                m = min(cands)
                chosen.append(m[1])
                cands.remove(m)
            rows.append([ry * W + rx] + chosen)
    return np.array(rows, dtype=np.int64)


CASES = [
    (1, 16, 16, 1, 7, 4),
    (1, 24, 20, 3, 9, 8),
    (3, 16, 16, 2, 7, 4),
    (3, 20, 18, 3, 9, 8),
    (1, 19, 17, 4, 11, 16),
]


@pytest.mark.parametrize("C,H,W,s,w,K", CASES)
def test_matches_brute_force(C, H, W, s, w, K):
    y = synth.tiny(10 + C + H + W, C, H, W, sigma=20.0)
    idx, dist, _ = matching.match(y, 8, s, w, K)
    np.testing.assert_array_equal(idx, brute_match(y, 8, s, w, K))
    assert np.all(np.diff(dist[:, 1:], axis=1) >= 0)


def test_forced_ties_constant_image():
    # Every distance is 0: slot 0 is the reference, the rest is the K-1
    # lowest indices of the window other than the reference.
    y = np.full((1, 16, 16), 77.25, dtype=np.float32)
    idx, dist, _ = matching.match(y, 8, 2, 5, 8)
    np.testing.assert_array_equal(idx, brute_match(y, 8, 2, 5, 8))
    assert not dist.any()
    ys, xs, _, _ = ref_grid(16, 16, 8, 2)
    for n, (ry, rx) in enumerate(zip(ys, xs)):
        y0, y1, x0, x1 = window(ry, rx, 9, 9, 5)
        exp = [a * 16 + b for a in range(y0, y1 + 1) for b in range(x0, x1 + 1)
               if (a, b) != (ry, rx)][:7]
        assert list(idx[n, 1:]) == exp


def test_forced_ties_clipped_plateau_sigma0():
    # A clean image clipped to [0, 255] has flat plateaus: many exact ties.
    clean = synth.clean_image(77, 0, 1, 24, 24, 30)
    y = np.clip(clean * 3.0, 0, 255).astype(np.float32)
    idx, _, _ = matching.match(y, 8, 3, 9, 8)
    np.testing.assert_array_equal(idx, brute_match(y, 8, 3, 9, 8))


def test_rgb_with_equal_channels_equals_gray():
    g = synth.tiny(5, 1, 20, 20, sigma=15.0)
    rgb = np.repeat(g, 3, axis=0)
    i1, _, _ = matching.match(g, 8, 3, 9, 8)
    i3, _, green = matching.match(rgb, 8, 3, 9, 8)
    assert green.all()
    np.testing.assert_array_equal(i1, i3)


def test_gcp_branch_boundary():
    # Reference patch with constant qG = 5 and qR = 6: gamma*||G|| = 1.2*5*8 = 48
    # = ||R|| exactly -> the >= of Eq. 10 selects green; qR = 7 does not.
    for qr, expect in ((6, True), (7, False)):
        y = np.zeros((3, 8, 8), dtype=np.float32)
        y[0] = qr / 256.0
        y[1] = 5 / 256.0
        y[2] = 1 / 256.0
        q = matching.quantize(y)
        got = matching.gcp_green(q, np.array([0]), np.array([0]), 8, 6, 5)
        assert bool(got[0]) is expect


def test_quantize_rounding_and_clamp():
    v = np.array([0.5, 1.5, 2.5, -0.5, -1.5, 3.0, 1e9, -1e9, np.nan, np.inf, -np.inf]) / 256.0
    q = matching.quantize(v.astype(np.float64))
    exp = [0, 2, 2, 0, -2, 3, 2 ** 20 - 1, -(2 ** 20 - 1), 0, 2 ** 20 - 1, -(2 ** 20 - 1)]
    assert list(q) == exp
    for a in np.random.default_rng(0).uniform(-300, 600, 200).astype(np.float32):
        assert matching.quantize(np.array([a]))[0] == _q(a)


def test_reference_grid_covers_every_pixel():
    for n, s in ((9, 3), (10, 3), (17, 8), (1, 2), (30, 4)):
        pos = ref_positions(n, s)
        assert pos[0] == 0 and pos[-1] == n - 1
        assert np.all(np.diff(pos) <= s) and np.all(np.diff(pos) > 0)
