"""Pins for the oracle's global basis and t-SVD projection
(Sec. II.C Eq. 3-7, Sec. III.B.1 Eq. 11-12, Eq. 18 and 20).

The t-product is checked against its definition through explicit block
circulant matrices (Eq. 3-4), which the oracle never builds.
"""
import numpy as np
import pytest

from oracle import basis, filtering
from paper_2508_10307_amd import synth


def bcirc(A):
    """Eq. 3: block (i, j) is the frontal slice (i - j) mod c.  A [c][n1][n2]."""
    c, n1, n2 = A.shape
    M = np.zeros((c * n1, c * n2))
    for i in range(c):
        for j in range(c):
            M[i * n1:(i + 1) * n1, j * n2:(j + 1) * n2] = A[(i - j) % c]
    return M


def first_block_column(M, c, n1):
    return np.stack([M[i * n1:(i + 1) * n1, :M.shape[1] // c] for i in range(c)])


@pytest.fixture(scope="module", params=[1, 3])
def learned(request):
    C = request.param
    y = synth.tiny(40 + C, C, 40, 36, sigma=20.0, n_blobs=8)
    UF, VF, U, V, eU, eV = basis.global_basis(y, 8, 3)
    P = basis.ref_patches(y, 8, 3)
    return C, y, P, UF, VF, U, V, eU, eV


def test_orthogonal_tensors_eq11(learned):
    C, _, _, _, _, U, V, _, _ = learned
    for T in (U, V):
        B = bcirc(T)
        np.testing.assert_allclose(B.T @ B, np.eye(8 * C), atol=1e-12)


def test_fourier_slices_unitary_and_conjugate_symmetric(learned):
    C, _, _, UF, VF, U, V, _, _ = learned
    for F, R in ((UF, U), (VF, V)):
        for f in range(C):
            np.testing.assert_allclose(F[f].conj().T @ F[f], np.eye(8), atol=1e-12)
            np.testing.assert_allclose(F[f], np.conj(F[(C - f) % C]), atol=1e-14)
        np.testing.assert_allclose(np.fft.fft(R, axis=0), F, atol=1e-12)


def test_tproduct_matches_bcirc_definition(learned):
    C, _, P, UF, VF, U, V, _, _ = learned
    for p in P[:5]:
        S = filtering.tsvd_forward(p, UF, VF)
        ref = first_block_column(bcirc(U).T @ bcirc(p) @ bcirc(V), C, 8)
        np.testing.assert_allclose(S, ref, atol=1e-9)
        back = filtering.tsvd_inverse(S, UF, VF)
        ref_b = first_block_column(bcirc(U) @ bcirc(S) @ bcirc(V).T, C, 8)
        np.testing.assert_allclose(back, ref_b, atol=1e-9)
        np.testing.assert_allclose(back, p, atol=1e-9)
        # Parseval: the projection is orthogonal on R^{8x8xc}
        assert abs(np.linalg.norm(S) - np.linalg.norm(p)) <= 1e-10 * np.linalg.norm(p)


def test_eigen_residuals_order_and_trace(learned):
    C, _, P, UF, VF, _, _, eU, eV = learned
    CU, CV = basis.covariances(P)
    Ph = np.fft.fft(P, axis=1)
    for f in range(C // 2 + 1):
        for Cm, F, ev in ((CU[f], UF, eU[f]), (CV[f], VF, eV[f])):
            nrm = np.linalg.norm(Cm)
            assert np.all(np.diff(ev) <= 1e-9 * nrm)
            for j in range(8):
                r = Cm @ F[f][:, j] - ev[j] * F[f][:, j]
                assert np.linalg.norm(r) <= 1e-12 * nrm
        energy = np.sum(np.abs(Ph[:, f]) ** 2)
        assert abs(eU[f].sum() - energy) <= 1e-10 * energy
        assert abs(eV[f].sum() - energy) <= 1e-10 * energy


def test_covariance_definition_by_loops():
    # C_U(f) = sum_i P_hat_i P_hat_i^H with P_hat from the explicit DFT sum.
    y = synth.tiny(3, 3, 16, 16, sigma=10.0)
    P = basis.ref_patches(y, 8, 4)
    CU, CV = basis.covariances(P)
    for f in range(2):
        cu = np.zeros((8, 8), complex)
        cv = np.zeros((8, 8), complex)
        for p in P:
            ph = sum(p[j] * np.exp(-2j * np.pi * f * j / 3) for j in range(3))
            cu += ph @ ph.conj().T
            cv += ph.conj().T @ ph
        np.testing.assert_allclose(CU[f], cu, rtol=1e-12, atol=1e-6)
        np.testing.assert_allclose(CV[f], cv, rtol=1e-12, atol=1e-6)


def test_phase_convention(learned):
    C, _, _, UF, VF, _, _, _, _ = learned
    for F in (UF, VF):
        for f in range(C // 2 + 1):
            for j in range(8):
                col = F[f][:, j]
                k = int(np.argmax(np.abs(col)))
                assert abs(col[k].imag) < 1e-14 and col[k].real > 0
                assert np.all(np.abs(col[:k]) < np.abs(col[k]))


def test_gray_basis_diagonalises_second_moments():
    # c = 1: U^T (sum P P^T) U and V^T (sum P^T P) V are diagonal, descending.
    y = synth.tiny(8, 1, 48, 40, sigma=25.0, n_blobs=10)
    _, _, U, V, _, _ = basis.global_basis(y, 8, 3)
    P = basis.ref_patches(y, 8, 3)[:, 0]
    A = sum(p @ p.T for p in P)
    B = sum(p.T @ p for p in P)
    for M, X in ((A, U[0]), (B, V[0])):
        D = X.T @ M @ X
        off = D - np.diag(np.diag(D))
        assert np.abs(off).max() <= 1e-10 * np.abs(D).max()
        assert np.all(np.diff(np.diag(D)) <= 0)
