"""GPU parity of the weighted aggregation (Eq. 2 with w_g = 1 / max(1, kept
coefficients of group g), hts_params.flags = HTS_FLAG_WEIGHTED) against the
FP64 oracle, through the C ABI.

Same protocol as the uniform denoise tests: the oracle re-runs with the
GPU's exported keep-masks (so both sides count the same kept coefficients
per group), reports every disagreement with its margin to tau, and the
pixel bar (1e-3 on the 0..255 scale) applies to that run.
"""
import numpy as np
import pytest
import torch

from oracle import pipeline as opipe
from paper_2508_10307_amd import api, synth

pytestmark = pytest.mark.gpu

PIX_TOL = 1e-3
DELTA_REL = 2e-4
WT = api.L.HTS_FLAG_WEIGHTED


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev())


def log(*a):
    print(*a, flush=True)


def parity_weighted(y, sigma, p, label):
    out, st = api.hts_denoise(T(y), sigma, p, save=True)
    torch.cuda.synchronize()
    C = y.shape[0]
    idx = st["idx"].cpu().numpy().astype(np.int64)
    masks = opipe.unpack_masks(st["masks"].cpu().numpy().view(np.uint32), len(idx), p.K, C)
    r = opipe.denoise(y, sigma, 8, p.stride, p.window, p.K, p.tau_mult, idx=idx,
                      U=st["U"].cpu().numpy(), V=st["V"].cpu().numpy(), mask=masks,
                      weighted=True)
    tau = p.tau_mult * sigma
    log(label, "overrides", r["n_override"], "max margin", r["max_override_margin"])
    assert r["max_override_margin"] <= DELTA_REL * max(tau, 1.0)
    err = np.abs(out.cpu().numpy() - r["out"]).max()
    log(label, "max |gpu - oracle| =", err)
    assert err <= PIX_TOL
    return out, r


@pytest.mark.parametrize("C,H,W,s,w,K", [(3, 48, 40, 3, 15, 16), (3, 64, 61, 2, 21, 32),
                                          (1, 40, 33, 3, 9, 8), (1, 45, 45, 4, 21, 64),
                                          (3, 37, 29, 3, 9, 2)])
def test_weighted_denoise_matches_oracle(C, H, W, s, w, K):
    y = synth.tiny(500 + H + W + C, C, H, W, sigma=20.0, n_blobs=6)
    p = api.Params(stride=s, window=w, K=K, flags=WT)
    out, r = parity_weighted(y, 20.0, p, f"weighted{C}x{H}x{W}")
    u = api.hts_denoise(T(y), 20.0, api.Params(stride=s, window=w, K=K))
    assert not torch.equal(out, u)     # the weights change the average


def test_weighted_batch_equals_single_and_is_reproducible():
    ys = [synth.tiny(61 + i, 3, 40 + 8 * i, 48, sigma=15.0 + 5 * i, n_blobs=5) for i in range(3)]
    sig = [15.0, 20.0, 25.0]
    p = api.Params(stride=3, window=11, K=16, flags=WT)
    xs = [T(y) for y in ys]
    outs = api.hts_denoise_batch(xs, sig, p)
    outs2 = api.hts_denoise_batch(xs, sig, p)
    for x, s, o, o2 in zip(xs, sig, outs, outs2):
        assert torch.equal(o, o2)
        assert torch.equal(o, api.hts_denoise(x, s, p))
    # other filter tile shapes give the same bits (integer sums)
    for shape in (1, 3, 5):
        q = api.Params(stride=3, window=11, K=16, flags=WT, tune=shape | (1 << 6))
        assert torch.equal(api.hts_denoise(xs[0], 15.0, q), outs[0])


def test_weighted_filter_num_and_weight_sums():
    """hts_filter with the flag adds weighted estimates into num and the
    weight sums into cnt; num / cnt is the weighted denoised image."""
    y = synth.tiny(73, 3, 40, 44, sigma=15.0)
    p = api.Params(stride=3, window=11, K=8, flags=WT)
    x = T(y)
    out, st = api.hts_denoise(x, 15.0, p, save=True)
    n_ref = st["idx"].shape[0]
    half = n_ref // 2
    a = api.hts_filter(x, 15.0, st["idx"], st["U"], st["V"], p, 0, half)
    b = api.hts_filter(x, 15.0, st["idx"], st["U"], st["V"], p, half, n_ref - half)
    num = (a["num"] + b["num"]).cpu().numpy()
    cnt = (a["cnt"] + b["cnt"]).cpu().numpy()
    assert np.abs(num / cnt[None] - out.cpu().numpy()).max() <= PIX_TOL
    idx = st["idx"].cpu().numpy().astype(np.int64)
    masks = opipe.unpack_masks(st["masks"].cpu().numpy().view(np.uint32), n_ref, 8, 3)
    r = opipe.denoise(y, 15.0, 8, 3, 11, 8, p.tau_mult, idx=idx, U=st["U"].cpu().numpy(),
                      V=st["V"].cpu().numpy(), mask=masks, weighted=True)
    np.testing.assert_allclose(cnt, r["cnt"], rtol=1e-5)


def test_zero_threshold_weighted_equals_uniform():
    """tau = 0 keeps every coefficient, so all groups weigh the same."""
    y = synth.tiny(88, 3, 40, 40, sigma=10.0)
    u = api.hts_denoise(T(y), 0.0, api.Params(stride=3, window=9, K=8))
    w = api.hts_denoise(T(y), 0.0, api.Params(stride=3, window=9, K=8, flags=WT))
    assert (u - w).abs().max().item() <= PIX_TOL


def test_weighted_unsupported_calls():
    y = synth.tiny(89, 1, 32, 32, sigma=10.0)
    p = api.Params(stride=3, window=9, K=8, flags=WT)
    x = T(y)
    num = torch.zeros_like(x)
    cnt = torch.zeros((32, 32), device=dev())
    with pytest.raises(api.L.HtsError):
        api.hts_aggregate(p, 1, 32, 32, num, cnt, out=torch.empty_like(x))
