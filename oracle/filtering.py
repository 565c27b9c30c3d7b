"""Collaborative filtering and aggregation (Sec. III.B.2, Eq. 18-20 and Eq. 2;
Alg. 1 Step 2(2)-(4) and Step 3).  Oracle, test infrastructure only."""
import numpy as np

from .haar import haar_matrix


def gather_groups(y: np.ndarray, idx: np.ndarray, ps: int) -> np.ndarray:
    """Stack the K patches of each group: [n_groups, K, C, ps, ps] float64."""
    C, H, W = y.shape
    y64 = np.asarray(y, dtype=np.float64)
    gy, gx = np.divmod(np.asarray(idx, dtype=np.int64), W)
    out = np.empty(idx.shape + (C, ps, ps), dtype=np.float64)
    for a in range(ps):
        for b in range(ps):
            out[..., a, b] = np.moveaxis(y64[:, gy + a, gx + b], 0, -1)
    return out


def tsvd_forward(P: np.ndarray, UF: np.ndarray, VF: np.ndarray) -> np.ndarray:
    """Patch-level projection U^T * P * V (t-product, Eq. 4-6 and 18).

    In the Fourier domain along the channel mode every frontal slice
    multiplies: S_hat(f) = UF(f)^H P_hat(f) VF(f); S is the inverse DFT,
    real because UF, VF are conjugate-symmetric in f.  P [..., C, ps, ps]."""
    Ph = np.fft.fft(P, axis=-3)
    Sh = np.conj(np.swapaxes(UF, -1, -2)) @ Ph @ VF
    return np.fft.ifft(Sh, axis=-3).real


def tsvd_inverse(S: np.ndarray, UF: np.ndarray, VF: np.ndarray) -> np.ndarray:
    """Inverse projection U * S * V^T (Eq. 20): P_hat(f) = UF(f) S_hat(f) VF(f)^H."""
    Sh = np.fft.fft(S, axis=-3)
    Ph = UF @ Sh @ np.conj(np.swapaxes(VF, -1, -2))
    return np.fft.ifft(Ph, axis=-3).real


def haar_group(T: np.ndarray, K: int) -> np.ndarray:
    """Group-mode transform x_4 U_Haar^T of Eq. 18 with U_group = U_Haar (Eq. 17).

    Reading: the coefficient along the group mode is H_K applied to the
    stack of K slot coefficients (slot order = distance order), i.e. row 0
    of H_K (the all-ones / sqrt(K) vector that Eq. 16 identifies with the
    dominant circulant eigenvector) gives the DC coefficient.  T [n, K, ...]."""
    H = haar_matrix(K)
    return np.einsum("kl,nl...->nk...", H, T)


def haar_group_inverse(S: np.ndarray, K: int) -> np.ndarray:
    """x_4 U_Haar^{-1} of Eq. 20; the Haar matrix is orthogonal, so H^{-1} = H^T."""
    H = haar_matrix(K)
    return np.einsum("lk,nl...->nk...", H, S)


def hard_threshold(S: np.ndarray, tau: float):
    """Eq. 19: keep S where |S| >= tau, zero elsewhere (DC included).
    Returns (S_truncate, keep-mask)."""
    keep = np.abs(S) >= tau
    return np.where(keep, S, 0.0), keep


def fourier_threshold(S: np.ndarray, tau: float, mask: np.ndarray = None):
    """Hard threshold in the channel-Fourier domain (reading F1; the paper
    thresholds the real core tensor, Eq. 19, and this variant keeps whole
    conjugate pairs, so it does not depend on a sign or phase convention).
    With F = DFT of S along the channel mode (c = 3): the f = 0 coefficient
    has orthonormal magnitude |F_0| / sqrt(3), the pair (f = 1, f = 2 =
    conj f = 1) the magnitude sqrt(2/3) |F_1| of its two real coordinates;
    each is kept iff its magnitude >= tau.  For c = 1 this is Eq. 19.
    S [..., C, ps, ps].  Returns (thresholded S, keep [..., C, ps, ps] with
    channel f holding the decision of frequency f, magnitudes a)."""
    C = S.shape[-3]
    if C == 1:
        a = np.abs(S)
        keep = a >= tau if mask is None else np.asarray(mask, dtype=bool)
        return np.where(keep, S, 0.0), keep, a
    assert C == 3
    F = np.fft.fft(S, axis=-3)
    a = np.empty(S.shape)
    a[..., 0, :, :] = np.abs(F[..., 0, :, :]) / np.sqrt(3.0)
    a[..., 1, :, :] = np.sqrt(2.0 / 3.0) * np.abs(F[..., 1, :, :])
    a[..., 2, :, :] = a[..., 1, :, :]
    if mask is None:
        keep = a >= tau
    else:
        mask = np.asarray(mask, dtype=bool)
        keep = np.stack([mask[..., 0, :, :], mask[..., 1, :, :], mask[..., 1, :, :]], axis=-3)
    return np.fft.ifft(np.where(keep, F, 0.0), axis=-3).real, keep, a


def aggregate(est: np.ndarray, idx: np.ndarray, C: int, H: int, W: int, ps: int,
              w: np.ndarray = None):
    """Step 3 / Eq. 2.  Uniform weights ("averagely written back", the
    default): num[p] = sum of all estimates covering p, cnt[p] = how many
    estimates cover p.  With per-group weights w [n] (Eq. 2's w, every patch
    of group g weighted w[g]): num[p] = sum w * estimate, cnt[p] = sum w.
    est [n, K, C, ps, ps], idx [n, K].  Returns (num [C,H,W], cnt [H,W])."""
    num = np.zeros(C * H * W, dtype=np.float64)
    cnt = np.zeros(H * W, dtype=np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    base = idx.ravel()
    wk = None if w is None else np.repeat(np.asarray(w, dtype=np.float64), idx.shape[1])
    for a in range(ps):
        for b in range(ps):
            pix = base + a * W + b
            cnt += np.bincount(pix, weights=wk, minlength=H * W)
            for ch in range(C):
                e = est[:, :, ch, a, b].ravel()
                num[ch * H * W:(ch + 1) * H * W] += np.bincount(
                    pix, weights=e if wk is None else wk * e, minlength=H * W)
    return num.reshape(C, H, W), cnt.reshape(H, W)


def group_weights(keep: np.ndarray) -> np.ndarray:
    """Reading W1 of Eq. 2's weights (the paper leaves them open; the
    BM3D-style choice): w_g = 1 / max(1, number of coefficients of group g
    kept by the hard threshold), over all K*C*ps*ps coefficients.
    keep [n, K, C, ps, ps] bool -> w [n]."""
    n = keep.reshape(keep.shape[0], -1).sum(axis=1)
    return 1.0 / np.maximum(n, 1).astype(np.float64)
