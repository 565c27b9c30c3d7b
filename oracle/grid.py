"""Reference grid and search windows (Alg. 1 Step 1) - oracle, test infrastructure only."""
import numpy as np


def ref_positions(n_valid: int, stride: int) -> np.ndarray:
    """Reference top-left coordinates along one axis.

    Reading (the paper is silent): 0, s, 2s, ... up to n_valid-1, plus
    n_valid-1 itself when the stride does not land on it, so that with
    s <= ps every pixel is covered by at least one reference patch.
    ``n_valid`` = H - ps + 1 (number of valid top-left rows).
    """
    pos = list(range(0, n_valid, stride))
    if pos[-1] != n_valid - 1:
        pos.append(n_valid - 1)
    return np.array(pos, dtype=np.int64)


def ref_grid(H: int, W: int, ps: int, stride: int):
    """(ys, xs) of all references in row-major order of the reference grid."""
    ry = ref_positions(H - ps + 1, stride)
    rx = ref_positions(W - ps + 1, stride)
    ys = np.repeat(ry, len(rx))
    xs = np.tile(rx, len(ry))
    return ys, xs, len(ry), len(rx)


def window(y: int, x: int, Hp: int, Wp: int, window_w: int):
    """Inclusive candidate range [y0, y1] x [x0, x1] for the reference at (y, x).

    Reading: ``window_w`` is the full (odd) width; radius r = (w-1)/2; at the
    image border the window is truncated to valid top-left positions (not
    shifted, not padded)."""
    r = (window_w - 1) // 2
    return max(0, y - r), min(Hp - 1, y + r), max(0, x - r), min(Wp - 1, x + r)
