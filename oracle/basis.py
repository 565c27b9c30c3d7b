"""Global circulant patch basis (Sec. III.B.1, Eq. 11-12; Alg. 1 Step 2(1)).

Oracle, test infrastructure only.
"""
import numpy as np

from .grid import ref_grid


def ref_patches(y: np.ndarray, ps: int, stride: int) -> np.ndarray:
    """All reference patches of the noisy image, [n_ref, C, ps, ps] float64
    (the paper uses all reference patches to avoid random sampling)."""
    C, H, W = y.shape
    ys, xs, _, _ = ref_grid(H, W, ps, stride)
    y64 = np.asarray(y, dtype=np.float64)
    return np.stack([y64[:, a:a + ps, b:b + ps] for a, b in zip(ys, xs)])


def normalize_phase(vecs: np.ndarray) -> np.ndarray:
    """Scale each column by a unit-modulus factor so that its entry of largest
    modulus is real and positive (first such entry on exact ties).

    Reading: eigenvectors are defined up to sign (real) or phase (complex);
    for c = 3 the real-domain coefficients depend on that choice, so one
    convention is fixed."""
    out = np.array(vecs, dtype=np.complex128, copy=True)
    for j in range(out.shape[1]):
        k = int(np.argmax(np.abs(out[:, j])))
        v = out[k, j]
        out[:, j] *= np.conj(v) / abs(v)
    return out


def covariances(P: np.ndarray):
    """Per-frequency second moments of the reference patches.

    P_hat(f) = sum_j P(:,:,j) exp(-2 pi i f j / c) (FFT along the channel
    mode, Eq. 6).  C_U(f) = sum_i P_hat_i(f) P_hat_i(f)^H and
    C_V(f) = sum_i P_hat_i(f)^H P_hat_i(f) for f = 0..floor(c/2), uncentred.

    Reading of Eq. 11-12: as printed the problem is degenerate (S_i is free),
    so the bases are taken as the two-sided nonlocal PCA of the t-SVD
    lineage the paper follows: in the Fourier domain of the t-product each
    frontal slice of U (V) is the eigenbasis of the row (column) second
    moment of the transformed patches."""
    n, C, ps = P.shape[0], P.shape[1], P.shape[2]
    Ph = np.fft.fft(P, axis=1)
    CU, CV = [], []
    for f in range(C // 2 + 1):
        X = Ph[:, f]                                   # [n, ps, ps]
        # the sums as one product each: R = [X_1 X_2 ... X_n] (side by side)
        # gives R R^H = sum X_i X_i^H; S = [X_1; X_2; ...; X_n] (stacked)
        # gives S^H S = sum X_i^H X_i
        R = np.moveaxis(X, 0, 1).reshape(ps, n * ps)
        S = X.reshape(n * ps, ps)
        CU.append(R @ R.conj().T)
        CV.append(S.conj().T @ S)
    return CU, CV


def basis_from_covariances(CU, CV, C: int):
    """Eigen-decompose each covariance (descending eigenvalues, phase
    convention of normalize_phase), extend to all frequencies by conjugate
    symmetry U_F(c-f) = conj(U_F(f)), and return

      UF, VF [C][ps][ps] complex (Fourier-domain slices, unitary per f),
      U, V   [C][ps][ps] real (U = IDFT of UF along the channel mode, the
             orthogonal tensor of Eq. 12),
      eigU, eigV [floor(c/2)+1][ps] descending eigenvalues.
    Pairing across frequencies is by descending rank (column j of every
    slice belongs to the j-th largest eigenvalue of its frequency)."""
    ps = CU[0].shape[0]
    UF = np.zeros((C, ps, ps), dtype=np.complex128)
    VF = np.zeros((C, ps, ps), dtype=np.complex128)
    eigU, eigV = [], []
    for f in range(C // 2 + 1):
        for Cm, F, ev in ((CU[f], UF, eigU), (CV[f], VF, eigV)):
            w, v = np.linalg.eigh(Cm)
            order = np.argsort(-w, kind="stable")
            ev.append(w[order])
            F[f] = normalize_phase(v[:, order])
    for f in range(C // 2 + 1, C):
        UF[f] = np.conj(UF[C - f])
        VF[f] = np.conj(VF[C - f])
    U = np.fft.ifft(UF, axis=0)
    V = np.fft.ifft(VF, axis=0)
    return UF, VF, U.real.copy(), V.real.copy(), np.array(eigU), np.array(eigV)


def global_basis(y: np.ndarray, ps: int, stride: int):
    """Alg. 1 Step 2(1): learn U, V from all reference patches of y."""
    P = ref_patches(y, ps, stride)
    CU, CV = covariances(P)
    return basis_from_covariances(CU, CV, y.shape[0])


def fourier_from_real(U: np.ndarray) -> np.ndarray:
    """UF = DFT of a real basis tensor along the channel mode (for overrides)."""
    return np.fft.fft(np.asarray(U, dtype=np.float64), axis=0)
