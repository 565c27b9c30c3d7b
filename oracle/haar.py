"""Haar matrix (Sec. II.D, Eq. 8-9) - oracle, test infrastructure only."""
import numpy as np


def haar_matrix(K: int) -> np.ndarray:
    """K x K Haar matrix, K a power of two >= 2.

    Eq. 8 gives H_2 = [[1, 1], [1, -1]] / sqrt(2); Eq. 9 builds
    H_2N = [H_N kron [1, 1]; I_N kron [1, -1]] / sqrt(2).
    Rows are the analysis vectors: row 0 is the all-ones vector / sqrt(K),
    which Eq. 16 identifies with the dominant eigenvector of circ(G)circ(G)^T.
    """
    if K < 2 or K & (K - 1):
        raise ValueError("K must be a power of two >= 2")
    H = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    n = 2
    while n < K:
        top = np.kron(H, np.array([[1.0, 1.0]]))
        bot = np.kron(np.eye(n), np.array([[1.0, -1.0]]))
        H = np.vstack([top, bot]) / np.sqrt(2.0)
        n *= 2
    return H
