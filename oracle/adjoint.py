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
multiplier enters only through the frozen mask, so its derivative is zero;
the relaxed mask of reading S1 (below) gives a surrogate derivative.
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


# ---------------------------------------------------------------- threshold gradient
# Reading S1 (a surrogate; the paper's hard threshold has a zero derivative
# almost everywhere): the keep-mask of Eq. 19 is relaxed to
#     m(s) = phi((|s| - tau) / eps),  phi = the logistic function,
# with width eps = kappa * sigma (kappa given), only to differentiate with
# respect to tau = lambda * sigma.  With grouping, basis and coverage count
# frozen, x_soft = diag(1/cnt) Place Q^T diag(m) Q Gather y, so for a loss L
# with gradient g = dL/dx_soft
#     dL/dtau = sum over groups and coefficients of r * s * dm/dtau,
#     s = Q Gather y,  r = Q Gather (g / cnt),  dm/dtau = -phi'(u) / eps,
# and dL/dlambda = sigma * dL/dtau.

def _logistic(u):
    return 0.5 * (1.0 + np.tanh(0.5 * u))


def soft_forward(y, idx, U, V, K, tau, eps, cnt, ps=8, chunk=2048):
    """x_soft for the relaxed mask (cnt = the frozen coverage count)."""
    y = np.asarray(y, dtype=np.float64)
    C, H, W = y.shape
    UF, VF = _basis.fourier_from_real(U), _basis.fourier_from_real(V)
    num = np.zeros((C, H, W))
    for c0 in range(0, len(idx), chunk):
        ic = idx[c0:c0 + chunk]
        S = _f.haar_group(_f.tsvd_forward(_f.gather_groups(y, ic, ps), UF, VF), K)
        St = _logistic((np.abs(S) - tau) / eps) * S
        est = _f.tsvd_inverse(_f.haar_group_inverse(St, K), UF, VF)
        nn, _ = _f.aggregate(est, ic, C, H, W, ps)
        num += nn
    return num / cnt[None]


def tau_gradient(y, g, idx, U, V, cnt, K, tau, eps, ps=8, chunk=2048, with_scale=False):
    """dL/dtau of reading S1 for the loss gradient g = dL/dx (sum over all
    groups of r * s * dm/dtau in the orthonormal Haar/t-SVD domain).  With
    with_scale, also the sum of the terms' magnitudes (a scale for
    comparisons)."""
    y = np.asarray(y, dtype=np.float64)
    r_img = np.asarray(g, dtype=np.float64) / cnt[None]
    UF, VF = _basis.fourier_from_real(U), _basis.fourier_from_real(V)
    total, scale = 0.0, 0.0
    for c0 in range(0, len(idx), chunk):
        ic = idx[c0:c0 + chunk]
        S = _f.haar_group(_f.tsvd_forward(_f.gather_groups(y, ic, ps), UF, VF), K)
        R = _f.haar_group(_f.tsvd_forward(_f.gather_groups(r_img, ic, ps), UF, VF), K)
        u = (np.abs(S) - tau) / eps
        ph = _logistic(u)
        terms = R * S * (-ph * (1.0 - ph) / eps)
        total += float(terms.sum())
        scale += float(np.abs(terms).sum())
    return (total, scale) if with_scale else total
