"""Pins of the derivative through the learned basis (reading B1) in the
oracle: each link of the chain against central finite differences of the
map it differentiates (the frozen-mask forward in U and V; the phase-fixed
eigenvectors in the matrix; the full y -> x_hat map with the basis learned
from y), and the scale invariance of the basis (<basis term, y> = 0)."""
import numpy as np
import pytest

from oracle import adjoint, basis, basis_adjoint as ba, pipeline


def _setup(C, H, W, K, seed):
    rng = np.random.default_rng(seed)
    y = rng.normal(100.0, 25.0, size=(C, H, W))
    r = pipeline.denoise(y, 20.0, ps=8, stride=3, window=9, K=K, return_mask=True)
    g = rng.normal(size=y.shape)
    return rng, y, r, g


@pytest.mark.parametrize("C,K", [(1, 8), (3, 4)])
def test_basis_cotangents_match_finite_differences(C, K):
    rng, y, r, g = _setup(C, 22, 20, K, 30 + C)
    idx, mask, U, V, cnt = r["idx"], r["mask"], r["U"], r["V"], r["cnt"]
    AU, AV = ba.basis_cotangents(y, g, idx, mask, U, V, cnt, K)
    gU, gV = np.fft.ifft(AU, axis=0), np.fft.ifft(AV, axis=0)
    assert np.abs(gU.imag).max() < 1e-9 * np.abs(gU).max()
    for which, grad in (("U", gU.real), ("V", gV.real)):
        d = rng.normal(size=U.shape)
        h = 1e-6

        def L(t):
            Uu = U + t * d if which == "U" else U
            Vv = V + t * d if which == "V" else V
            return float((g * adjoint.frozen_forward(y, idx, mask, Uu, Vv, K)[0]).sum())

        fd = (L(h) - L(-h)) / (2 * h)
        assert float((grad * d).sum()) == pytest.approx(fd, rel=1e-6)


def _phase_eigvecs(Cm):
    w, v = np.linalg.eigh(Cm)
    order = np.argsort(-w, kind="stable")
    return basis.normalize_phase(v[:, order]), w[order]


@pytest.mark.parametrize("complex_", [False, True])
def test_eig_vjp_matches_finite_differences(complex_):
    rng = np.random.default_rng(7 + complex_)
    X = rng.normal(size=(8, 40)) + (1j * rng.normal(size=(8, 40)) if complex_ else 0)
    Cm = X @ X.conj().T
    G = rng.normal(size=(8, 8)) + (1j * rng.normal(size=(8, 8)) if complex_ else 0)
    vecs, vals = _phase_eigvecs(Cm)
    Cb = ba.eig_vjp(vecs, vals, G)
    np.testing.assert_allclose(Cb, Cb.conj().T, atol=1e-14)
    E = rng.normal(size=(8, 8)) + (1j * rng.normal(size=(8, 8)) if complex_ else 0)
    dC = E + E.conj().T
    h = 1e-6
    L = lambda t: float(np.real(np.vdot(G, _phase_eigvecs(Cm + t * dC)[0])))
    fd = (L(h) - L(-h)) / (2 * h)
    assert float(np.real(np.trace(Cb @ dC))) == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_gauge_term_matters_for_complex_eigenvectors():
    # without the phase term the complex case misses the derivative of the
    # normalisation (a dropped term must fail the pin above)
    rng = np.random.default_rng(9)
    X = rng.normal(size=(8, 40)) + 1j * rng.normal(size=(8, 40))
    vecs, vals = _phase_eigvecs(X @ X.conj().T)
    G = rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8))
    Wm = vecs.conj().T @ G
    F = np.array([[0.0 if j == k else 1.0 / (vals[k] - vals[j]) for k in range(8)]
                  for j in range(8)])
    Cb = vecs @ (F * Wm) @ vecs.conj().T
    assert np.abs(0.5 * (Cb + Cb.conj().T) - ba.eig_vjp(vecs, vals, G)).max() > 1e-8 * np.abs(Cb).max()


@pytest.mark.parametrize("C,K", [(1, 8), (3, 4)])
def test_full_gradient_matches_finite_differences(C, K):
    rng, y, r, g = _setup(C, 20, 19, K, 40 + C)
    idx, mask, cnt = r["idx"], r["mask"], r["cnt"]
    frozen = adjoint.frozen_adjoint(g, idx, mask, r["U"], r["V"], cnt, K)
    term = ba.basis_term(y, g, idx, mask, K)
    total = frozen + term
    h = 1e-5
    d = rng.normal(size=y.shape)
    L = lambda t: ba.basis_loss(y + t * d, g, idx, mask, cnt, K)
    fd = (L(h) - L(-h)) / (2 * h)
    assert float((total * d).sum()) == pytest.approx(fd, rel=1e-6)
    # the basis term is not negligible: the frozen adjoint alone misses it
    assert abs(float((term * d).sum())) > 1e-4 * abs(fd)
    for (ch, a, b) in [(0, 0, 0), (C - 1, 7, 11), (0, 19, 18), (C - 1, 10, 3)]:
        e = np.zeros_like(y)
        e[ch, a, b] = 1.0
        hp = 1e-3      # one pixel moves L by little: a wider step keeps rounding out
        fdp = (ba.basis_loss(y + hp * e, g, idx, mask, cnt, K)
               - ba.basis_loss(y - hp * e, g, idx, mask, cnt, K)) / (2 * hp)
        assert total[ch, a, b] == pytest.approx(fdp, rel=1e-5, abs=1e-7)


@pytest.mark.parametrize("C,K", [(1, 8), (3, 4)])
def test_basis_term_is_orthogonal_to_y(C, K):
    # U(alpha y) = U(y): moving y along itself leaves the basis unchanged
    _, y, r, g = _setup(C, 21, 22, K, 50 + C)
    term = ba.basis_term(y, g, r["idx"], r["mask"], K)
    assert abs(float((term * y).sum())) < 1e-8 * np.abs(term).sum() * np.abs(y).max()
