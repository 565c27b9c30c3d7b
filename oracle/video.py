"""Video denoising with spatio-temporal patch search (Sec. IV, real-world
colour video: the patch search runs over the spatial and the temporal
dimension) - oracle, test infrastructure only.

Reading V1 (the paper gives no more detail):
  * frames y[t] (t < T) share C, H, W; each frame has the reference grid of
    Alg. 1 Step 1 (grid.ref_grid); references are numbered frame by frame,
    row-major within a frame;
  * the candidates of a reference at (t, i, j) are all valid positions
    (t', i', j') with |t' - t| <= dt (truncated at the ends of the sequence)
    and (i', j') in the truncated spatial window of grid.window;
  * distances are the exact integer distances of matching.match on the
    guide of the reference's frame (GCP branch from the reference patch for
    c = 3, the band mean for other c), applied to the candidate frame's guide
    plane of the same kind;
  * positions are numbered in the stacked image of the T frames one above
    the other ([C][T*H][W]): idx = (t' H + i') W + j'; slot 0 is the
    reference, the other slots the K-1 smallest (distance, idx);
  * one basis for the whole sequence, from the reference patches of every
    frame (Eq. 11-12 over their union); the groups are filtered as in
    Eq. 18-20 and averaged (Eq. 2) over the stacked image, whose patches
    never straddle two frames.
With T = 1 or dt = 0 the matching is that of each frame on its own.
"""
import numpy as np

from . import basis as _basis
from . import filtering as _f
from . import matching as _m
from .grid import ref_grid, window


def stack(frames: np.ndarray) -> np.ndarray:
    """[T][C][H][W] -> the stacked image [C][T*H][W]."""
    T, C, H, W = frames.shape
    return np.ascontiguousarray(np.transpose(frames, (1, 0, 2, 3)).reshape(C, T * H, W))


def unstack(img: np.ndarray, T: int) -> np.ndarray:
    C, TH, W = img.shape
    return np.ascontiguousarray(np.transpose(img.reshape(C, T, TH // T, W), (1, 0, 2, 3)))


def match(frames: np.ndarray, ps: int, stride: int, window_w: int, K: int, dt: int,
          gcp_num: int = 6, gcp_den: int = 5):
    """Spatio-temporal top-K grouping.  Returns (idx [T*n_ref, K] int64 in
    stacked coordinates, dist [T*n_ref, K] int64)."""
    T, C, H, W = frames.shape
    Hp, Wp = H - ps + 1, W - ps + 1
    ys, xs, _, _ = ref_grid(H, W, ps, stride)
    planes, green = [], []
    for t in range(T):
        q = _m.quantize(frames[t])
        planes.append(_m.guide_planes(q))
        green.append(_m.gcp_green(q, ys, xs, ps, gcp_num, gcp_den))
    n_ref = len(ys)
    idx = np.zeros((T * n_ref, K), dtype=np.int64)
    dist = np.zeros((T * n_ref, K), dtype=np.int64)
    for t in range(T):
        for n in range(n_ref):
            ry, rx = int(ys[n]), int(xs[n])
            plane = 0 if (C != 3 or green[t][n]) else 1
            ref = planes[t][plane][ry:ry + ps, rx:rx + ps]
            y0, y1, x0, x1 = window(ry, rx, Hp, Wp, window_w)
            ds, cs = [], []
            for t2 in range(max(0, t - dt), min(T - 1, t + dt) + 1):
                g = planes[t2][plane]
                for i in range(y0, y1 + 1):
                    for j in range(x0, x1 + 1):
                        if t2 == t and i == ry and j == rx:
                            continue
                        ds.append(int(((g[i:i + ps, j:j + ps] - ref) ** 2).sum()))
                        cs.append((t2 * H + i) * W + j)
            if len(ds) < K - 1:
                raise ValueError("window holds fewer than K candidates")
            ds, cs = np.array(ds, dtype=np.int64), np.array(cs, dtype=np.int64)
            order = np.lexsort((cs, ds))[:K - 1]
            r = t * n_ref + n
            idx[r, 0] = (t * H + ry) * W + rx
            idx[r, 1:] = cs[order]
            dist[r, 1:] = ds[order]
    return idx, dist


def global_basis(frames: np.ndarray, ps: int, stride: int):
    """One basis for the sequence: Eq. 11-12 over the reference patches of
    every frame (basis.basis_from_covariances of the summed moments)."""
    T, C = frames.shape[:2]
    P = np.concatenate([_basis.ref_patches(frames[t], ps, stride) for t in range(T)])
    CU, CV = _basis.covariances(P)
    return _basis.basis_from_covariances(CU, CV, C)


def denoise(frames, sigma, ps=8, stride=3, window=21, K=16, dt=1, tau_mult=2.7, idx=None,
            U=None, V=None, mask=None, chunk=2048):
    """Video Haar-tSVD.  frames [T][C][H][W].  Overrides (idx, U, V, mask) as
    in pipeline.denoise.  Returns dict(out [T][C][H][W], idx, U, V, cnt
    (stacked [T*H][W]), n_override, max_override_margin)."""
    frames = np.asarray(frames, dtype=np.float64)
    T, C, H, W = frames.shape
    if idx is None:
        idx, _ = match(frames, ps, stride, window, K, dt)
    if U is None:
        UF, VF, U, V, _, _ = global_basis(frames, ps, stride)
    else:
        U = np.asarray(U, dtype=np.float64)
        V = np.asarray(V, dtype=np.float64)
        UF, VF = _basis.fourier_from_real(U), _basis.fourier_from_real(V)
    y = stack(frames)
    tau = float(tau_mult) * float(sigma)
    num = np.zeros((C, T * H, W))
    cnt = np.zeros((T * H, W))
    n_over, max_margin = 0, 0.0
    for c0 in range(0, len(idx), chunk):
        ic = idx[c0:c0 + chunk]
        S = _f.haar_group(_f.tsvd_forward(_f.gather_groups(y, ic, ps), UF, VF), K)
        St, keep = _f.hard_threshold(S, tau)
        if mask is not None:
            mk = np.asarray(mask[c0:c0 + chunk], dtype=bool)
            diff = mk != keep
            if diff.any():
                n_over += int(diff.sum())
                max_margin = max(max_margin, float(np.abs(np.abs(S[diff]) - tau).max()))
            St = np.where(mk, S, 0.0)
        est = _f.tsvd_inverse(_f.haar_group_inverse(St, K), UF, VF)
        nn, cc = _f.aggregate(est, ic, C, T * H, W, ps)
        num += nn
        cnt += cc
    return {"out": unstack(num / cnt[None], T), "idx": idx, "U": U, "V": V, "cnt": cnt,
            "n_override": n_over, "max_override_margin": max_margin}
