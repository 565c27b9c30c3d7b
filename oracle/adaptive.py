"""A-Haar-tSVD noise-level adjustment (Sec. III.D, Eq. 21-22; Algorithm
A-Haar-tSVD) - oracle, test infrastructure only.

The CNN estimator of the paper is out of scope: the caller supplies sigma_est.
What is built is the eigenvalue test that adjusts it.

Readings (the paper leaves these open):
  A1  circ(G) is the block circulant of the group along its group mode: for a
      group of K patches p_1..p_K (each flattened to d = c*ps*ps values), the
      column j of circ(G) stacks p_{1-j}, ..., p_{K-j} (indices mod K).  Its
      K x K Gram matrix circ(G)^T circ(G) is circulant and has the same
      nonzero eigenvalues as circ(G) circ(G)^T; they are
      lambda_m = sum over the d values of |DFT_K(p_1..p_K)[m]|^2, m = 0..K-1,
      and lambda_{K/2} is the value Eq. 21 names lambda-hat (the alternating
      vector is the DFT's K/2 mode).
  A2  a = the rank of lambda-hat among the K eigenvalues in ascending order,
      1-based, counting the eigenvalues strictly below it
      (a = 1 + #{m : lambda_m < lambda-hat}).
  A3  the sampled groups are given by the caller as reference indices (the
      random draw of the paper is an input here); the majority vote adjusts
      sigma when more than half of the sampled groups have a <= gamma
      (a tie keeps sigma_est).
  A4  sub-images are independent images: each is matched, gets its own
      global basis and is filtered with its own sigma-hat (Algorithm
      A-Haar-tSVD, Step 2); they tile the image without overlap.
"""
import numpy as np

from . import filtering as _f
from . import matching as _m
from . import pipeline as _p


def circulant_eigenvalues(G: np.ndarray) -> np.ndarray:
    """lambda_m, m = 0..K-1, of circ(G)^T circ(G) for one group G [K, ...]
    (reading A1): the DFT along the group mode, squared moduli summed over
    every other index."""
    G = np.asarray(G, dtype=np.float64).reshape(G.shape[0], -1)
    F = np.fft.fft(G, axis=0)
    return (F.real ** 2 + F.imag ** 2).sum(axis=1)


def rank_position(lams: np.ndarray) -> int:
    """Reading A2: 1-based ascending rank of lambda_{K/2} among the K values."""
    lams = np.asarray(lams, dtype=np.float64)
    K = lams.shape[0]
    return 1 + int((lams < lams[K // 2]).sum())


def group_ranks(y: np.ndarray, idx: np.ndarray, samples, ps: int = 8) -> np.ndarray:
    """Rank a (Eq. 22) of every sampled group: idx [n_ref, K] match indices
    (slot order: distance to the reference), samples = reference indices."""
    samples = np.asarray(samples, dtype=np.int64)
    G = _f.gather_groups(y, np.asarray(idx, dtype=np.int64)[samples], ps)
    return np.array([rank_position(circulant_eigenvalues(g)) for g in G], dtype=np.int64)


def adjust_sigma(ranks, sigma_est: float, beta: float = 1.2, gamma: int = 13) -> float:
    """Eq. 22 with the majority vote over the sampled groups (reading A3)."""
    ranks = np.asarray(ranks)
    votes = int((ranks <= gamma).sum())
    return float(sigma_est) / float(beta) if 2 * votes > ranks.shape[0] else float(sigma_est)


def a_haar_tsvd(y, sigma_est, subs, samples, ps=8, stride=3, window=21, K=16,
                tau_mult=2.7, beta=1.2, gamma=13, gcp_num=6, gcp_den=5):
    """Algorithm A-Haar-tSVD: for each sub-image (y0, x0, h, w) of subs, the
    matching of Algorithm 1 Step 1, the ranks of its sampled groups
    (samples[i] = reference indices of sub-image i), sigma-hat by Eq. 22, then
    Haar-tSVD of the sub-image with sigma-hat (reading A4).  Returns the
    stitched estimate and the per-sub-image sigma-hat and ranks."""
    y = np.asarray(y)
    out = np.zeros(y.shape, dtype=np.float64)
    sig, rk = [], []
    for (y0, x0, h, w), smp in zip(subs, samples):
        sub = np.ascontiguousarray(y[:, y0:y0 + h, x0:x0 + w])
        idx, _, _ = _m.match(sub, ps, stride, window, K, gcp_num, gcp_den)
        ranks = group_ranks(sub, idx, smp, ps)
        s_hat = adjust_sigma(ranks, sigma_est, beta, gamma)
        res = _p.denoise(sub, s_hat, ps, stride, window, K, tau_mult, gcp_num, gcp_den, idx=idx)
        out[:, y0:y0 + h, x0:x0 + w] = res["out"]
        sig.append(s_hat)
        rk.append(ranks)
    return out, sig, rk
