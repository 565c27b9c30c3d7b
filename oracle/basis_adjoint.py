"""Derivative of the denoiser through its learned basis (adjoint extension,
reading B1) - oracle, test infrastructure only.

The frozen adjoint holds U and V fixed, but Alg. 1 Step 2(1) learns them
from the noisy image itself (Eq. 11-12 read as the per-frequency
eigenproblems of the patch second moments), so with grouping, keep-masks
and coverage count frozen the full derivative of x_hat adds a term through
U(y), V(y).  With g = dL/dx_hat, r = g / cnt and, per group slot,
P = the gathered patch of y, R = that of r,

  T  = U^T * P * V              (t-product projection, Eq. 18)
  T' = H^T M H T                (Haar along the group, frozen mask, inverse)
  D  = H^T M H (U^T * R * V)    (dL/dT)

the cotangents of the real basis tensors are (the t-product algebra keeps
<A * B, C> = <A, C * B^T>):

  dL/dU = sum over slots of  R * V * T'^T + P * V * D^T
  dL/dV = sum over slots of  R^T * U * T' + P^T * U * D

In the Fourier domain of the channel mode these are, per frequency f,
A_U(f) = sum R^(f) V_F(f) T'^(f)^H + P^(f) V_F(f) D^(f)^H and
A_V(f) = sum R^(f)^H U_F(f) T'^(f) + P^(f)^H U_F(f) D^(f).

U_F(f) for f = 0..floor(c/2) are the phase-normalised eigenvectors of
C_U(f) = sum_i P^_i(f) P^_i(f)^H (descending), the rest conjugates, and
U = IDFT(U_F); so dL/dU_F(f) = (w_f / c) A_U(f) with w_f = 1 for the real
frequencies (f = 0, and f = c/2 for even c) and 2 for the others.  Through
the eigen-decomposition (first-order perturbation of a Hermitian
eigenproblem with distinct eigenvalues) and the phase convention (the
largest-modulus entry u_m of each eigenvector stays real positive):

  G~ = G + i (Im <G_k, u_k> / u_m) e_m   per column k   (gauge term)
  Cbar = U (F o (U^H G~)) U^H,  F_jk = 1 / (lambda_k - lambda_j), F_kk = 0

and only the Hermitian part of Cbar matters.  Finally C_U(f) = sum P^P^H
and C_V(f) = sum P^^H P^ give dL/dP^_i(f) = 2 Cbar_U(f) P^_i(f)
+ 2 P^_i(f) Cbar_V(f) for every reference patch, and
dL/dP_i(:,:,j) = sum over f <= c/2 of Re(dL/dP^_i(f) e^{2 pi i f j / c})
is added back at the reference's position.
"""
import numpy as np

from . import basis as _basis
from . import filtering as _f
from .grid import ref_grid


def basis_cotangents(y, g, idx, mask, U, V, cnt, K, ps=8, chunk=2048):
    """(A_U, A_V) [C][ps][ps] complex for every frequency f = 0..C-1: the
    Fourier-domain cotangents of the real basis tensors, dL/dU = IDFT(A_U)
    (real), for L with gradient g = dL/dx_hat of the frozen-mask map
    x_hat(y; U, V)."""
    y = np.asarray(y, dtype=np.float64)
    C, H, W = y.shape
    UF, VF = _basis.fourier_from_real(U), _basis.fourier_from_real(V)
    r = np.asarray(g, dtype=np.float64) / cnt[None]
    AU = np.zeros((C, ps, ps), dtype=np.complex128)
    AV = np.zeros((C, ps, ps), dtype=np.complex128)
    herm = lambda X: np.conj(np.swapaxes(X, -1, -2))
    for c0 in range(0, len(idx), chunk):
        ic = idx[c0:c0 + chunk]
        m = mask[c0:c0 + chunk]
        P = _f.gather_groups(y, ic, ps)
        R = _f.gather_groups(r, ic, ps)
        Tp = _f.haar_group_inverse(np.where(m, _f.haar_group(_f.tsvd_forward(P, UF, VF), K), 0.0), K)
        D = _f.haar_group_inverse(np.where(m, _f.haar_group(_f.tsvd_forward(R, UF, VF), K), 0.0), K)
        Ph, Rh = np.fft.fft(P, axis=-3), np.fft.fft(R, axis=-3)
        Tph, Dh = np.fft.fft(Tp, axis=-3), np.fft.fft(D, axis=-3)
        AU += (Rh @ VF @ herm(Tph) + Ph @ VF @ herm(Dh)).sum(axis=(0, 1))
        AV += (herm(Rh) @ UF @ Tph + herm(Ph) @ UF @ Dh).sum(axis=(0, 1))
    return AU, AV


def eig_vjp(vecs, vals, G):
    """Cotangent of a Hermitian matrix C from the cotangent G (dL = Re <G, dU>,
    <a, b> = sum conj(a) b) of its phase-normalised eigenvectors U = vecs
    (columns, largest-modulus entry real positive) with distinct eigenvalues
    vals: the Hermitian matrix Cbar_h with dL = Re tr(Cbar_h dC)."""
    U = np.asarray(vecs, dtype=np.complex128)
    n = U.shape[0]
    Gt = np.array(G, dtype=np.complex128, copy=True)
    for k in range(n):
        m = int(np.argmax(np.abs(U[:, k])))
        Gt[m, k] += 1j * np.imag(np.vdot(Gt[:, k], U[:, k])) / U[m, k].real
    Wm = U.conj().T @ Gt
    lam = np.asarray(vals, dtype=np.float64)
    F = np.zeros((n, n))
    for j in range(n):
        for k in range(n):
            if j != k:
                F[j, k] = 1.0 / (lam[k] - lam[j])
    Cb = U @ (F * Wm) @ U.conj().T
    return 0.5 * (Cb + Cb.conj().T)


def frequency_weights(C):
    """w_f / c for f = 0..floor(c/2): dL/dU_F(f) = (w_f / c) A_U(f)."""
    return np.array([(1.0 if (f == 0 or 2 * f == C) else 2.0) / C for f in range(C // 2 + 1)])


def covariance_cotangents(y, g, idx, mask, K, ps=8, stride=3):
    """(Cbar_U(f), Cbar_V(f)) for f = 0..floor(c/2), with the basis learned
    from y itself (Alg. 1 Step 2(1))."""
    C = y.shape[0]
    UF, VF, U, V, eigU, eigV = _basis.global_basis(y, ps, stride)
    cnt = _f.aggregate(np.zeros((len(idx), K, C, ps, ps)), idx, C, y.shape[1], y.shape[2], ps)[1]
    AU, AV = basis_cotangents(y, g, idx, mask, U, V, cnt, K, ps)
    wf = frequency_weights(C)
    CbU = [eig_vjp(UF[f], eigU[f], wf[f] * AU[f]) for f in range(C // 2 + 1)]
    CbV = [eig_vjp(VF[f], eigV[f], wf[f] * AV[f]) for f in range(C // 2 + 1)]
    return CbU, CbV


def basis_term(y, g, idx, mask, K, ps=8, stride=3):
    """The part of dL/dy that flows through U(y), V(y) (reading B1), to be
    added to the frozen adjoint D^T g."""
    y = np.asarray(y, dtype=np.float64)
    C, H, W = y.shape
    CbU, CbV = covariance_cotangents(y, g, idx, mask, K, ps, stride)
    ys, xs, _, _ = ref_grid(H, W, ps, stride)
    P = _basis.ref_patches(y, ps, stride)
    Ph = np.fft.fft(P, axis=1)
    j = np.arange(C)
    dP = np.zeros_like(P)
    for f in range(C // 2 + 1):
        Gf = 2.0 * (CbU[f] @ Ph[:, f] + Ph[:, f] @ CbV[f])       # [n_ref, ps, ps]
        tw = np.exp(2j * np.pi * f * j / C)                      # e^{2 pi i f j / c}
        dP += np.real(Gf[:, None] * tw[None, :, None, None])
    out = np.zeros((C, H, W))
    for i, (a, b) in enumerate(zip(ys, xs)):
        out[:, a:a + ps, b:b + ps] += dP[i]
    return out


def basis_loss(y, g, idx, mask, cnt, K, ps=8, stride=3):
    """L(y) = <g, x_hat(y)> with grouping, masks and count frozen and the
    basis learned from y: the function whose gradient is the frozen adjoint
    plus basis_term (used by the finite-difference pins)."""
    from .adjoint import _group_operator
    y = np.asarray(y, dtype=np.float64)
    C, H, W = y.shape
    UF, VF, _, _, _, _ = _basis.global_basis(y, ps, stride)
    num = np.zeros((C, H, W))
    for c0 in range(0, len(idx), 2048):
        ic = idx[c0:c0 + 2048]
        est = _group_operator(_f.gather_groups(y, ic, ps), UF, VF, mask[c0:c0 + 2048], K)
        num += _f.aggregate(est, ic, C, H, W, ps)[0]
    return float((np.asarray(g, dtype=np.float64) * num / cnt[None]).sum())
