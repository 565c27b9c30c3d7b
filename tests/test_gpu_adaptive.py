"""GPU parity of the A-Haar-tSVD noise-level adjustment (Sec. III.D, Eq. 21-22)
through the C ABI against the FP64 oracle.

Bar: the rank of every sampled group and the voted sigma-hat are exact (the
ranks are integers decided in FP64 on both sides; sigma-hat is sigma_est or
the float32 quotient sigma_est / beta).  The adaptive batch must then give
bit for bit the output of the plain batch run with those sigma-hat values,
whose parity with the oracle is covered by the denoise tests; one sub-image
is checked against the oracle here as well.
"""
import numpy as np
import pytest
import torch

from oracle import adaptive as oad
from oracle import matching as omatch
from oracle import pipeline as opipe
from paper_2508_10307_amd import api, synth

pytestmark = pytest.mark.gpu


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev())


def log(*a):
    print(*a, flush=True)


def sigma_hat_f32(ranks, sigma_est, beta, gamma):
    votes = int((np.asarray(ranks) <= gamma).sum())
    if 2 * votes > len(ranks):
        return np.float32(np.float32(sigma_est) / np.float32(beta))
    return np.float32(sigma_est)


@pytest.mark.parametrize("C,H,W,s,w,K,sigma", [(3, 48, 44, 3, 15, 16, 25.0),
                                                (3, 56, 52, 3, 21, 32, 10.0),
                                                (1, 40, 36, 3, 11, 8, 30.0),
                                                (1, 45, 45, 4, 21, 64, 15.0),
                                                (3, 30, 28, 3, 9, 4, 20.0)])
def test_ranks_and_sigma_match_oracle(C, H, W, s, w, K, sigma):
    y = synth.tiny(900 + H + W + C, C, H, W, sigma=sigma, n_blobs=6)
    idx_o, _, _ = omatch.match(y, 8, s, w, K)
    n_ref = idx_o.shape[0]
    smp = np.random.default_rng(H * W + K).choice(n_ref, size=min(24, n_ref), replace=False)
    p = api.Params(stride=s, window=w, K=K)
    log("case", C, H, W, s, w, K, "samples", len(smp))
    sig, ranks = api.hts_adapt_sigma(T(y), torch.from_numpy(idx_o.astype(np.int32)).to(dev()),
                                     smp.astype(np.int32), sigma, p)
    torch.cuda.synchronize()
    r_o = oad.group_ranks(y, idx_o, smp)
    np.testing.assert_array_equal(ranks.cpu().numpy(), r_o)
    assert sig.item() == sigma_hat_f32(r_o, sigma, 1.2, 13)
    assert sig.item() == pytest.approx(oad.adjust_sigma(r_o, sigma), rel=1e-6)
    log("ranks", r_o.tolist(), "sigma-hat", sig.item())


def test_constant_image_votes_for_the_adjustment():
    """Identical patches: lambda_{K/2} = 0 is the smallest eigenvalue (a = 1)."""
    y = np.full((3, 40, 40), 77.0)
    p = api.Params(stride=3, window=9, K=16)
    idx = api.hts_match(T(y), p)
    sig, ranks = api.hts_adapt_sigma(T(y), idx, np.arange(10, dtype=np.int32), 24.0, p,
                                     beta=1.5, gamma=1)
    assert ranks.cpu().numpy().tolist() == [1] * 10
    assert sig.item() == np.float32(np.float32(24.0) / np.float32(1.5))


def test_invalid_arguments_are_rejected():
    p = api.Params(stride=3, window=9, K=8)
    x = T(np.zeros((1, 24, 24)))
    idx = torch.zeros(64 * 8, dtype=torch.int32, device=dev())
    with pytest.raises(api.L.HtsError):
        api.hts_adapt_sigma(x, idx, np.zeros(4, dtype=np.int32), 10.0, p, beta=0.0)
    with pytest.raises(api.L.HtsError):
        api.hts_adapt_sigma(x, idx, np.zeros(4, dtype=np.int32), -1.0, p)


def test_adaptive_batch_equals_plain_batch_with_sigma_hat_and_oracle():
    """Two sub-images of one picture: sigma-hat and ranks against the oracle
    (on the GPU's own indices, which the match tests pin to the oracle's),
    the output bit-equal to the plain batch with those sigma-hat, and one
    sub-image against the oracle's Haar-tSVD with its sigma-hat."""
    y = synth.tiny(4242, 3, 64, 96, sigma=20.0, n_blobs=8)
    p = api.Params(stride=3, window=15, K=16)
    subs = api.sub_images(64, 96, 64, 48)
    assert subs == [(0, 0, 64, 48), (0, 48, 64, 48)]
    smp = api.draw_samples(subs, p, 16, seed=3)
    parts = [T(y[:, y0:y0 + h, x0:x0 + w]) for (y0, x0, h, w) in subs]
    outs, sig, ranks = api.hts_denoise_batch_adaptive(parts, [20.0, 20.0], smp, p)
    torch.cuda.synchronize()
    sig = sig.cpu().numpy()
    _, so, ro = oad.a_haar_tsvd(y, 20.0, subs, smp, 8, 3, 15, 16)
    for i in range(2):
        np.testing.assert_array_equal(ranks[i].cpu().numpy(), ro[i])
        assert sig[i] == sigma_hat_f32(ro[i], 20.0, 1.2, 13)
        assert sig[i] == pytest.approx(so[i], rel=1e-6)
    log("sigma-hat", sig.tolist(), "ranks", [r.tolist() for r in ro])
    plain = api.hts_denoise_batch(parts, [float(v) for v in sig], p)
    for a, b in zip(outs, plain):
        assert torch.equal(a, b)
    # the oracle's Haar-tSVD of the first sub-image with its sigma-hat
    out1, st = api.hts_denoise(parts[0], float(sig[0]), p, save=True)
    assert torch.equal(out1, outs[0])
    sub0 = y[:, :64, :48]
    idx = st["idx"].cpu().numpy().astype(np.int64)
    masks = opipe.unpack_masks(st["masks"].cpu().numpy().view(np.uint32), len(idx), 16, 3)
    r = opipe.denoise(sub0, float(sig[0]), 8, 3, 15, 16, p.tau_mult, idx=idx,
                      U=st["U"].cpu().numpy(), V=st["V"].cpu().numpy(), mask=masks)
    assert r["max_override_margin"] <= 2e-4 * max(p.tau_mult * float(sig[0]), 1.0)
    err = np.abs(outs[0].cpu().numpy() - r["out"]).max()
    log("sub-image 0 max |gpu - oracle| =", err)
    assert err <= 1e-3


def test_adaptive_graph_replays_take_new_samples_and_sigma():
    """The captured batch graph reads samples, sigma_est and the output slots
    from the descriptor table: replays with other inputs give fresh results,
    and a plain batch of the same shapes is a separate graph."""
    y = synth.tiny(77, 3, 48, 48, sigma=15.0, n_blobs=5)
    p = api.Params(stride=3, window=11, K=8)
    x = [T(y)]
    n_ref = np.prod(api.ref_grid(48, 48, p))
    s1 = np.arange(0, 12, dtype=np.int32).reshape(1, -1)
    s2 = (n_ref - 1 - np.arange(0, 12, dtype=np.int32)).reshape(1, -1)
    o1, g1, r1 = api.hts_denoise_batch_adaptive(x, [15.0], s1, p)
    o2, g2, r2 = api.hts_denoise_batch_adaptive(x, [40.0], s2, p)
    torch.cuda.synchronize()
    idx = api.hts_match(x[0], p)
    for smp, sg, g, r in ((s1, 15.0, g1, r1), (s2, 40.0, g2, r2)):
        gs, rs = api.hts_adapt_sigma(x[0], idx, smp, sg, p)
        assert torch.equal(r[0], rs)
        assert g[0].item() == gs.item()
    plain = api.hts_denoise_batch(x, [float(g2[0])], p)
    assert torch.equal(plain[0], o2[0])
    assert not torch.equal(o1[0], o2[0])
