"""Algorithm 1 (Haar-tSVD) end to end - oracle, test infrastructure only.

Step 1 grouping (matching.match), Step 2(1) global basis (basis.global_basis),
Step 2(2)-(4) forward transform, hard threshold, inverse (filtering), Step 3
averaged write-back (filtering.aggregate).  Optional overrides let a parity
test feed in match indices, a basis or threshold masks produced elsewhere and
check everything downstream of them.
"""
import numpy as np

from . import basis as _basis
from . import filtering as _f
from . import matching as _m


def unpack_masks(words: np.ndarray, n: int, K: int, C: int, ps: int = 8) -> np.ndarray:
    """Bit-packed keep-masks (bit ((g*K+k)*C+ch)*ps*ps + a*ps + b of a little-
    endian uint32 stream) -> bool [n, K, C, ps, ps]."""
    bits = np.unpackbits(np.ascontiguousarray(words, dtype="<u4").view(np.uint8),
                         bitorder="little")
    return bits[: n * K * C * ps * ps].astype(bool).reshape(n, K, C, ps, ps)


def denoise(y, sigma, ps=8, stride=3, window=21, K=16, tau_mult=2.7, gcp_num=6,
            gcp_den=5, idx=None, U=None, V=None, mask=None, return_mask=False,
            chunk=2048, weighted=False, fourier=False):
    """Denoise y [C][H][W] with noise level sigma.

    idx      optional [n_ref, K] match indices (else Step 1 is run here);
    U, V     optional real basis tensors [C][ps][ps] (else Step 2(1));
    mask     optional bool keep-mask [n_ref, K, C, ps, ps] used instead of the
             oracle's own Eq. 19 decision; every position where it disagrees
             is reported with the oracle's margin | |S| - tau |.
    weighted Eq. 2 with the group weights of filtering.group_weights (from
             the keep-mask in use) instead of uniform ones.
    fourier  threshold in the channel-Fourier domain (filtering.
             fourier_threshold) instead of Eq. 19 on the real core tensor;
             masks then hold the decision of frequency f in channel f.
    Returns a dict with out (= num / cnt), num, cnt, idx, U, V, UF, VF, and,
    when asked, the oracle's keep-mask and the override report."""
    y = np.asarray(y)
    C, H, W = y.shape
    res = {}
    if idx is None:
        idx, dist, green = _m.match(y, ps, stride, window, K, gcp_num, gcp_den)
        res["dist"], res["green"] = dist, green
    idx = np.asarray(idx, dtype=np.int64)
    if U is None:
        UF, VF, U, V, eU, eV = _basis.global_basis(y, ps, stride)
        res["eigU"], res["eigV"] = eU, eV
    else:
        U = np.asarray(U, dtype=np.float64)
        V = np.asarray(V, dtype=np.float64)
        UF, VF = _basis.fourier_from_real(U), _basis.fourier_from_real(V)
    tau = float(tau_mult) * float(sigma)
    num = np.zeros((C, H, W))
    cnt = np.zeros((H, W))
    own_masks = [] if return_mask else None
    n_over, max_margin, over_margins = 0, 0.0, []
    for c0 in range(0, len(idx), chunk):
        ic = idx[c0:c0 + chunk]
        G = _f.gather_groups(y, ic, ps)
        S = _f.haar_group(_f.tsvd_forward(G, UF, VF), K)
        if fourier:
            St, keep, mag = _f.fourier_threshold(S, tau)
        else:
            St, keep = _f.hard_threshold(S, tau)
            mag = np.abs(S)
        if return_mask:
            own_masks.append(keep)
        if mask is not None:
            mk = np.asarray(mask[c0:c0 + chunk], dtype=bool)
            if fourier:
                St, mk, _ = _f.fourier_threshold(S, tau, mk)
            else:
                St = np.where(mk, S, 0.0)
            diff = mk != keep
            if diff.any():
                marg = np.abs(mag[diff] - tau)
                n_over += int(diff.sum())
                max_margin = max(max_margin, float(marg.max()))
                over_margins.append(marg)
            keep = mk
        est = _f.tsvd_inverse(_f.haar_group_inverse(St, K), UF, VF)
        wg = _f.group_weights(keep) if weighted else None
        nn, cc = _f.aggregate(est, ic, C, H, W, ps, wg)
        num += nn
        cnt += cc
    res.update(out=num / cnt[None], num=num, cnt=cnt, idx=idx, U=U, V=V, UF=UF, VF=VF,
               tau=tau)
    if return_mask:
        res["mask"] = np.concatenate(own_masks)
    if mask is not None:
        res["n_override"] = n_over
        res["max_override_margin"] = max_margin
        res["override_margins"] = (np.concatenate(over_margins) if over_margins
                                   else np.zeros(0))
    return res


def group_coefficients(y, idx, U, V, K, ps=8):
    """S_noisy of Eq. 18 for the given groups (rows of idx), [n, K, C, ps, ps]."""
    UF, VF = _basis.fourier_from_real(U), _basis.fourier_from_real(V)
    G = _f.gather_groups(np.asarray(y), np.asarray(idx, dtype=np.int64), ps)
    return _f.haar_group(_f.tsvd_forward(G, UF, VF), K)
