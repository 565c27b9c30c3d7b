"""GPU parity of the surrogate threshold derivative (hts_denoise_grad_tau,
reading S1: logistic relaxation of the keep-mask, width kappa * sigma) with
the FP64 oracle, on the oracle's own grouping and basis (the basis rounded to
float32 on both sides, as the GPU takes it).  Bar: the difference is below
2e-3 of sigma * (sum of the terms' magnitudes)."""
import numpy as np
import pytest
import torch

from oracle import adjoint as oadj
from oracle import pipeline as opipe
from paper_2508_10307_amd import api, synth

pytestmark = pytest.mark.gpu


def dev():
    return torch.device("cuda:0")


def T(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(dev())


def log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("C,H,W,s,w,K,kappa", [(1, 32, 30, 3, 9, 8, 0.1), (3, 40, 36, 3, 11, 16, 0.2),
                                                (3, 36, 36, 3, 11, 32, 0.05), (1, 30, 28, 2, 7, 4, 0.5)])
def test_grad_tau_matches_oracle(C, H, W, s, w, K, kappa):
    sigma = 20.0
    y = synth.tiny(950 + H + C, C, H, W, sigma=sigma, n_blobs=5)
    r = opipe.denoise(y, sigma, 8, s, w, K, 2.7)
    U32, V32 = r["U"].astype(np.float32), r["V"].astype(np.float32)
    g = np.random.default_rng(H * W).normal(size=y.shape)
    ana, scale = oadj.tau_gradient(y, g, r["idx"], U32.astype(np.float64), V32.astype(np.float64),
                                   r["cnt"], K, 2.7 * sigma, kappa * sigma, with_scale=True)
    st = {"idx": T(r["idx"], np.int32), "U": T(U32), "V": T(V32), "cnt": T(r["cnt"])}
    p = api.Params(stride=s, window=w, K=K, tau_mult=2.7)
    gt = api.hts_denoise_grad_tau(T(y), T(g), st, sigma, p, kappa).item()
    gt2 = api.hts_denoise_grad_tau(T(y), T(g), st, sigma, p, kappa).item()
    log("gpu", gt, "oracle", sigma * ana, "scale", sigma * scale)
    assert gt == gt2
    assert abs(gt - sigma * ana) <= 2e-3 * sigma * scale
    assert abs(sigma * ana) > 1e-3 * sigma * scale     # a non-trivial case


def test_autograd_returns_the_surrogate_tau_gradient():
    y = synth.tiny(977, 3, 40, 40, sigma=15.0)
    clean = synth.clean_image(977, 0, 3, 40, 40, 4)
    p = api.Params(stride=3, window=11, K=8)
    x = T(y)
    lam = torch.tensor(2.7, dtype=torch.float32, device=dev(), requires_grad=True)
    out = api.HaarTSVD.apply(x, 15.0, lam, p, 0.1)
    loss = ((out - T(clean)) ** 2).mean()
    loss.backward()
    g = 2.0 * (out.detach() - T(clean)) / out.numel()
    _, st = api.hts_denoise(x, 15.0, p, save=True)
    ref = api.hts_denoise_grad_tau(x, g, st, 15.0, p, 0.1)
    assert lam.grad.item() == pytest.approx(ref.item(), rel=1e-6)
    assert lam.grad.item() != 0.0
    # without a relaxation width the exact (zero) derivative stays
    lam2 = torch.tensor(2.7, dtype=torch.float32, device=dev(), requires_grad=True)
    api.HaarTSVD.apply(x, 15.0, lam2, p).sum().backward()
    assert lam2.grad.item() == 0.0


def test_grad_tau_edge_cases():
    y = synth.tiny(978, 1, 24, 24, sigma=10.0)
    p = api.Params(stride=3, window=9, K=8)
    x = T(y)
    _, st = api.hts_denoise(x, 10.0, p, save=True)
    assert api.hts_denoise_grad_tau(x, torch.ones_like(x), st, 0.0, p, 0.1).item() == 0.0
    with pytest.raises(api.L.HtsError):
        api.hts_denoise_grad_tau(x, torch.ones_like(x), st, 10.0, p, 0.0)
