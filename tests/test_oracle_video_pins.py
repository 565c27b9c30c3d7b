"""Pins of the video oracle's sequence basis and spatio-temporal matcher
(reading V1 of Sec. IV: one basis for the whole sequence from Eq. 11-12
over the reference patches of every frame; candidates from frames
t - dt .. t + dt in the truncated spatial window), against definitions
written out here independently of oracle.video / oracle.basis:

* the sequence basis must diagonalise, per channel frequency, the second
  moments summed over every frame's reference patches, each DFT written as
  its explicit sum and each reference position from its own loop (not
  grid.ref_grid); its eigenvalues are those diagonals and their traces are
  the summed patch energies;
* the basis of a sequence does not depend on the order of its frames and
  differs from the basis of any single frame;
* a pure-Python exhaustive matcher (exact Fraction rounding, big-integer
  distances, repeated minimum extraction over every frame of the temporal
  reach) reproduces video.match on a translating clip with dt > 0.

Each pin is also run against a deliberately broken copy of the oracle
function (planted here, on the CPU) to show that it fails on the mistake
it is meant to catch."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import basis, video
from paper_2508_10307_amd import synth


def _axis_refs(n_valid, s):
    out, v = [], 0
    while v < n_valid:
        out.append(v)
        v += s
    if out[-1] != n_valid - 1:
        out.append(n_valid - 1)
    return out


def _summed_moments_by_loops(frames, ps, s):
    """C_U(f), C_V(f) of Eq. 11-12 summed over every frame's reference
    patches, with P_hat(f) = sum_j P(:,:,j) exp(-2 pi i f j / c) spelled out."""
    T, C, H, W = frames.shape
    nf = C // 2 + 1
    CU = [np.zeros((ps, ps), complex) for _ in range(nf)]
    CV = [np.zeros((ps, ps), complex) for _ in range(nf)]
    energy = [0.0] * nf
    for t in range(T):
        for ry in _axis_refs(H - ps + 1, s):
            for rx in _axis_refs(W - ps + 1, s):
                P = frames[t, :, ry:ry + ps, rx:rx + ps].astype(np.float64)
                for f in range(nf):
                    ph = sum(P[j] * np.exp(-2j * np.pi * f * j / C) for j in range(C))
                    CU[f] += ph @ ph.conj().T
                    CV[f] += ph.conj().T @ ph
                    energy[f] += float((np.abs(ph) ** 2).sum())
    return CU, CV, energy


def _check_sequence_basis(frames, ps, s, result):
    """True when (UF, VF, eU, eV) diagonalise the summed moments of every
    frame, descending, with eigenvalues equal to the diagonals."""
    UF, VF, _, _, eU, eV = result
    CU, CV, energy = _summed_moments_by_loops(frames, ps, s)
    C = frames.shape[1]
    for f in range(C // 2 + 1):
        for M, F, ev in ((CU[f], UF[f], eU[f]), (CV[f], VF[f], eV[f])):
            D = F.conj().T @ M @ F
            scale = np.abs(M).max()
            off = D - np.diag(np.diag(D))
            if np.abs(off).max() > 1e-10 * scale:
                return False
            if np.abs(np.diag(D).real - ev).max() > 1e-10 * scale:
                return False
            if np.any(np.diff(ev) > 1e-10 * scale):
                return False
            if abs(ev.sum() - energy[f]) > 1e-10 * energy[f]:
                return False
    return True


def _clip(T, C, H, W, seed, sigma=15.0):
    clean = synth.clean_video(seed, T, C, H, W, 5, motion=(1, 2))
    return np.stack([synth.add_awgn(seed, t, clean[t], sigma) for t in range(T)])


@pytest.mark.parametrize("C", [1, 3])
def test_sequence_basis_diagonalises_every_frames_moments(C):
    f = _clip(3, C, 20, 22, 800 + C)
    assert _check_sequence_basis(f, 8, 3, video.global_basis(f, 8, 3))


def test_sequence_basis_pin_catches_dropped_frames(monkeypatch):
    """A planted mistake: the sequence basis from frame 0 alone."""
    f = _clip(3, 3, 20, 22, 810)

    def first_frame_only(frames, ps, stride):
        return basis.global_basis(frames[0], ps, stride)

    monkeypatch.setattr(video, "global_basis", first_frame_only)
    assert not _check_sequence_basis(f, 8, 3, video.global_basis(f, 8, 3))


def test_sequence_basis_is_frame_order_invariant_and_not_one_frames():
    f = _clip(3, 3, 20, 22, 820)
    UF, VF, _, _, eU, eV = video.global_basis(f, 8, 3)
    UFr, VFr, _, _, eUr, eVr = video.global_basis(f[::-1].copy(), 8, 3)
    # summation order differs: agreement to rounding of the largest eigenvalue
    np.testing.assert_allclose(eUr, eU, rtol=0, atol=1e-12 * eU.max())
    np.testing.assert_allclose(eVr, eV, rtol=0, atol=1e-12 * eV.max())
    # same eigenvectors under the same phase convention (distinct eigenvalues)
    np.testing.assert_allclose(UFr, UF, atol=1e-8)
    np.testing.assert_allclose(VFr, VF, atol=1e-8)
    for t in range(3):
        e1 = basis.global_basis(f[t], 8, 3)[4]
        assert np.abs(e1 - eU).max() > 1e-3 * np.abs(eU).max()


def _q(v):
    x = Fraction(float(v)) * 256
    fl = x.numerator // x.denominator
    rem = x - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return max(-(2 ** 20 - 1), min(2 ** 20 - 1, fl))


def brute_video_match(frames, ps, s, w, K, dt, num=6, den=5):
    """Exhaustive spatio-temporal grouping in Python integers (reading V1)."""
    T, C, H, W = frames.shape
    q = [[[[_q(frames[t, c, i, j]) for j in range(W)] for i in range(H)] for c in range(C)]
         for t in range(T)]
    Hp, Wp = H - ps + 1, W - ps + 1
    r = (w - 1) // 2

    def g(t, kind, i, j):
        if C == 1:
            return q[t][0][i][j]
        if kind == "G":
            return q[t][1][i][j]
        return q[t][0][i][j] + q[t][1][i][j] + q[t][2][i][j]

    rows = []
    for t in range(T):
        for ry in _axis_refs(Hp, s):
            for rx in _axis_refs(Wp, s):
                kind = "G"
                if C == 3:
                    n2 = [sum(q[t][c][ry + a][rx + b] ** 2 for a in range(ps) for b in range(ps))
                          for c in range(3)]
                    kind = "G" if Fraction(num, den) ** 2 * n2[1] >= max(n2[0], n2[2]) else "S"
                cands = []
                for t2 in range(max(0, t - dt), min(T - 1, t + dt) + 1):
                    for cy in range(max(0, ry - r), min(Hp - 1, ry + r) + 1):
                        for cx in range(max(0, rx - r), min(Wp - 1, rx + r) + 1):
                            if (t2, cy, cx) == (t, ry, rx):
                                continue
                            d = 0
                            for a in range(ps):
                                for b in range(ps):
                                    e = g(t, kind, ry + a, rx + b) - g(t2, kind, cy + a, cx + b)
                                    d += e * e
                            cands.append((d, (t2 * H + cy) * W + cx))
                chosen = []
                for _ in range(K - 1):
                    m = min(cands)
                    chosen.append(m[1])
                    cands.remove(m)
                rows.append([(t * H + ry) * W + rx] + chosen)
    return np.array(rows, dtype=np.int64)


@pytest.mark.parametrize("C,dt,K", [(1, 1, 8), (3, 1, 8), (3, 2, 16)])
def test_video_match_equals_brute_force_on_a_translating_clip(C, dt, K):
    f = _clip(3, C, 16, 17, 830 + C + dt)
    idx, dist = video.match(f, 8, 3, 7, K, dt)
    np.testing.assert_array_equal(idx, brute_video_match(f, 8, 3, 7, K, dt))
    assert np.all(np.diff(dist[:, 1:], axis=1) >= 0)
    # the translation makes the other frames compete: some groups use them
    H, W = f.shape[2], f.shape[3]
    frame_of = idx // (H * W)
    ref_frame = idx[:, :1] // (H * W)
    assert (frame_of[:, 1:] != ref_frame).any()


def test_video_match_pin_catches_a_dropped_temporal_reach(monkeypatch):
    """A planted mistake: the matcher ignores the temporal reach."""
    f = _clip(3, 1, 16, 17, 840)
    real = video.match

    def no_reach(frames, ps, stride, window_w, K, dt, gcp_num=6, gcp_den=5):
        return real(frames, ps, stride, window_w, K, 0, gcp_num, gcp_den)

    monkeypatch.setattr(video, "match", no_reach)
    idx, _ = video.match(f, 8, 3, 7, 8, 1)
    assert not np.array_equal(idx, brute_video_match(f, 8, 3, 7, 8, 1))
