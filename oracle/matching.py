"""Grouping: GCP-guided block matching (Sec. III.A, Eq. 10; Alg. 1 Step 1).

Oracle, test infrastructure only.  Distances are exact integers, so the
ranking is exact and independent of summation order.
"""
import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

from .grid import ref_grid, window

QSCALE = 256.0          # guide grid: multiples of 1/256 grey level
QMAX = (1 << 20) - 1    # clamp of the quantised guide


def quantize(y: np.ndarray) -> np.ndarray:
    """Fixed-point guide q = round_half_even(256 * y), clamped to |q| <= 2^20 - 1.

    Reading: Eq. 10 compares Euclidean norms of patches; computing them on a
    1/256 grid makes every distance an exact integer (< 2^52), so the ranking
    of candidates has one correct answer regardless of arithmetic order.
    NaN maps to 0 and +-inf to the clamp.  256*y is exact for float32 y.
    """
    q = np.rint(np.asarray(y, dtype=np.float64) * QSCALE)
    q = np.where(np.isnan(q), 0.0, q)
    return np.clip(q, -QMAX, QMAX).astype(np.int64)


def band_mean(q: np.ndarray) -> np.ndarray:
    """The mean of the quantised bands on the same grid, rounded half to
    even, in exact integer arithmetic: round(sum_j q_j / c)."""
    c = q.shape[0]
    s = q.sum(axis=0)
    fl = np.floor_divide(s, c)
    r = s - fl * c                       # 0 <= r < c
    up = (2 * r > c) | ((2 * r == c) & (fl % 2 == 1))
    return fl + up.astype(np.int64)


def guide_planes(q: np.ndarray):
    """Guide planes from the quantised channels [C][H][W].

    c = 1: the channel itself.  c = 3: (G, R+G+B).  The channel sum is three
    times the RGB average of Eq. 10 and ranks candidates identically.

    Reading H1 (other band counts, the spectral tubes of HSI): the GCP test
    of Eq. 10 is an RGB rule and the paper names no matching guide for other
    band counts, so the guide is the band mean (band_mean), a choice of this
    oracle and of the kernels (the paper's HSI extension, Sec. III.E, uses
    the mean of the medium-wavelength bands for noise estimation, not for
    matching); it stays on the 2^-8 grid within the clamp, so distances stay
    exact integers."""
    if q.shape[0] == 1:
        return [q[0]]
    if q.shape[0] != 3:
        return [band_mean(q)]
    return [q[1], q[0] + q[1] + q[2]]


def gcp_green(q: np.ndarray, ys, xs, ps: int, num: int, den: int) -> np.ndarray:
    """Eq. 10 branch test for each reference patch (True = green-channel distance).

    Green is used when ||P^G|| >= max(||P^R||, ||P^B||) / gamma, gamma = num/den,
    evaluated on the reference patch only.  Squared and cleared of the
    fraction: num^2 * ||qG||^2 >= den^2 * max(||qR||^2, ||qB||^2), exact in int64."""
    out = np.zeros(len(ys), dtype=bool)
    if q.shape[0] != 3:
        return out
    for n, (y, x) in enumerate(zip(ys, xs)):
        nr = int((q[0, y:y + ps, x:x + ps] ** 2).sum())
        ng = int((q[1, y:y + ps, x:x + ps] ** 2).sum())
        nb = int((q[2, y:y + ps, x:x + ps] ** 2).sum())
        out[n] = num * num * ng >= den * den * max(nr, nb)
    return out


def match(y: np.ndarray, ps: int, stride: int, window_w: int, K: int,
          gcp_num: int = 6, gcp_den: int = 5):
    """Top-K grouping for every reference patch.

    Returns (idx [n_ref, K] int64, dist [n_ref, K] int64, green [n_ref] bool).
    idx = y*W + x of the top-left corner.  Readings:
      * slot 0 is the reference itself (distance 0; the paper sorts the group
        by distance to the reference, Sec. III.D);
      * slots 1..K-1 are the K-1 other candidates with the smallest
        (distance, idx), ties broken towards the lower idx (paper silent);
      * the candidate set is the truncated window of grid.window;
      * distance = sum over the patch of (g_ref - g_cand)^2 on the guide plane
        chosen by the reference's GCP branch (the square of Eq. 10's norm,
        same order).
    """
    C, H, W = y.shape
    Hp, Wp = H - ps + 1, W - ps + 1
    ys, xs, _, _ = ref_grid(H, W, ps, stride)
    q = quantize(y)
    planes = guide_planes(q)
    green = gcp_green(q, ys, xs, ps, gcp_num, gcp_den)
    views = [sliding_window_view(p, (ps, ps)) for p in planes]
    n_ref = len(ys)
    idx = np.zeros((n_ref, K), dtype=np.int64)
    dist = np.zeros((n_ref, K), dtype=np.int64)
    for n in range(n_ref):
        ry, rx = int(ys[n]), int(xs[n])
        plane = 0 if (C != 3 or green[n]) else 1
        v = views[plane]
        ref = v[ry, rx]
        y0, y1, x0, x1 = window(ry, rx, Hp, Wp, window_w)
        cand = v[y0:y1 + 1, x0:x1 + 1]
        d = ((cand - ref) ** 2).sum(axis=(2, 3)).ravel()
        cy, cx = np.meshgrid(np.arange(y0, y1 + 1), np.arange(x0, x1 + 1), indexing="ij")
        cidx = (cy * W + cx).ravel()
        keep = cidx != ry * W + rx
        d, cidx = d[keep], cidx[keep]
        if len(d) < K - 1:
            raise ValueError("window holds fewer than K candidates")
        order = np.lexsort((cidx, d))[:K - 1]
        idx[n, 0] = ry * W + rx
        idx[n, 1:] = cidx[order]
        dist[n, 1:] = d[order]
    return idx, dist, green
