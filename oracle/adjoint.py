"""Adjoint of the denoiser with frozen grouping, masks and basis - oracle,
test infrastructure only.

With the match indices, the Eq. 19 keep-masks, the basis U, V and the
coverage count held fixed, Eq. 18-20 and the averaged write-back (Eq. 2) make
x_hat a linear function of y:

    x_hat = D y = diag(1/cnt) Place Q^T M Q Gather y,

Gather stacks each group's patches, Q = (Haar along the group) o (t-SVD
projection) is orthogonal, M applies the frozen mask, Place adds each
estimate back at its position.  Its transpose, written step by step, is

    D^T z = Place Q^T M Q Gather diag(1/cnt) z

(Place^T = Gather, Gather^T = Place, (Q^T M Q)^T = Q^T M Q).  The threshold
multiplier enters only through the frozen mask, so its derivative is zero.
"""
import numpy as np

from . import basis as _basis
from . import filtering as _f


def _group_operator(G, UF, VF, mask, K):
    """Q^T M Q on stacked groups G [n, K, C, ps, ps]."""
    S = _f.haar_group(_f.tsvd_forward(G, UF, VF), K)
    S = np.where(mask, S, 0.0)
    return _f.tsvd_inverse(_f.haar_group_inverse(S, K), UF, VF)


def frozen_forward(y, idx, mask, U, V, K, ps=8, chunk=2048):
    """D y for the frozen map.  Returns (x_hat [C,H,W], cnt [H,W])."""
    y = np.asarray(y, dtype=np.float64)
    C, H, W = y.shape
    UF, VF = _basis.fourier_from_real(U), _basis.fourier_from_real(V)
    num = np.zeros((C, H, W))
    cnt = np.zeros((H, W))
    for c0 in range(0, len(idx), chunk):
        ic = idx[c0:c0 + chunk]
        est = _group_operator(_f.gather_groups(y, ic, ps), UF, VF, mask[c0:c0 + chunk], K)
        nn, cc = _f.aggregate(est, ic, C, H, W, ps)
        num += nn
        cnt += cc
    return num / cnt[None], cnt


def frozen_adjoint(z, idx, mask, U, V, cnt, K, ps=8, chunk=2048):
    """D^T z: scale by 1/cnt, gather (the transpose of Place), apply the
    symmetric group operator, place-add (the transpose of Gather)."""
    z = np.asarray(z, dtype=np.float64)
    C, H, W = z.shape
    UF, VF = _basis.fourier_from_real(U), _basis.fourier_from_real(V)
    r = z / cnt[None]
    out = np.zeros((C, H, W))
    for c0 in range(0, len(idx), chunk):
        ic = idx[c0:c0 + chunk]
        est = _group_operator(_f.gather_groups(r, ic, ps), UF, VF, mask[c0:c0 + chunk], K)
        nn, _ = _f.aggregate(est, ic, C, H, W, ps)
        out += nn
    return out


def mse_loss_grad(x_hat, clean, idx, mask, U, V, cnt, K, n_total, ps=8):
    """Gradient of L = sum((x_hat - clean)^2) / n_total with respect to the
    noisy input, through the frozen map: D^T (2 (x_hat - clean) / n_total)."""
    g = 2.0 * (np.asarray(x_hat, dtype=np.float64) - clean) / n_total
    return frozen_adjoint(g, idx, mask, U, V, cnt, K, ps)
