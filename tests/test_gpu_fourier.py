"""GPU parity of the channel-Fourier magnitude threshold (HTS_FLAG_FOURIER_THRESHOLD;
reading F1: f = 0 kept iff |F_0|/sqrt 3 >= tau, the conjugate pair f = 1, 2
iff sqrt(2/3)|F_1| >= tau) against the FP64 oracle, with the exported masks
(frequency f in channel f) re-applied by the oracle; pixel bar 1e-3."""
import numpy as np
import pytest
import torch

from oracle import pipeline as opipe
from paper_2508_10307_amd import api, synth

pytestmark = pytest.mark.gpu

PIX_TOL = 1e-3
DELTA_REL = 2e-4
FT = api.L.HTS_FLAG_FOURIER_THRESHOLD
WT = api.L.HTS_FLAG_WEIGHTED


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.device("cuda:0"))


def log(*a):
    print(*a, flush=True)


def parity(y, sigma, p, weighted, label):
    out, st = api.hts_denoise(T(y), sigma, p, save=True)
    torch.cuda.synchronize()
    C = y.shape[0]
    idx = st["idx"].cpu().numpy().astype(np.int64)
    masks = opipe.unpack_masks(st["masks"].cpu().numpy().view(np.uint32), len(idx), p.K, C)
    np.testing.assert_array_equal(masks[:, :, 1], masks[:, :, 2])   # pairs kept whole
    r = opipe.denoise(y, sigma, 8, p.stride, p.window, p.K, p.tau_mult, idx=idx,
                      U=st["U"].cpu().numpy(), V=st["V"].cpu().numpy(), mask=masks,
                      weighted=weighted, fourier=True)
    tau = p.tau_mult * sigma
    log(label, "overrides", r["n_override"], "max margin", r["max_override_margin"])
    assert r["max_override_margin"] <= DELTA_REL * max(tau, 1.0)
    assert r["n_override"] <= max(3, 1e-5 * masks.size)
    err = np.abs(out.cpu().numpy() - r["out"]).max()
    log(label, "max |gpu - oracle| =", err)
    assert err <= PIX_TOL
    return out


@pytest.mark.parametrize("H,W,s,w,K", [(48, 40, 3, 15, 16), (64, 61, 2, 21, 32), (37, 29, 3, 9, 2),
                                        (40, 44, 3, 11, 8)])
def test_fourier_threshold_matches_oracle(H, W, s, w, K):
    y = synth.tiny(700 + H + W, 3, H, W, sigma=20.0, n_blobs=6)
    out = parity(y, 20.0, api.Params(stride=s, window=w, K=K, flags=FT), False, f"ft{H}x{W}K{K}")
    assert not torch.equal(out, api.hts_denoise(T(y), 20.0, api.Params(stride=s, window=w, K=K)))


def test_fourier_threshold_weighted_matches_oracle():
    y = synth.tiny(801, 3, 48, 48, sigma=25.0, n_blobs=6)
    parity(y, 25.0, api.Params(stride=3, window=15, K=16, flags=FT | WT), True, "ft+w")


def test_gray_ignores_the_flag_and_batch_equals_single():
    g = synth.tiny(802, 1, 40, 36, sigma=15.0)
    assert torch.equal(api.hts_denoise(T(g), 15.0, api.Params(stride=3, window=9, K=8, flags=FT)),
                       api.hts_denoise(T(g), 15.0, api.Params(stride=3, window=9, K=8)))
    ys = [synth.tiny(803 + i, 3, 40 + 8 * i, 44, sigma=20.0) for i in range(2)]
    p = api.Params(stride=3, window=11, K=16, flags=FT)
    outs = api.hts_denoise_batch([T(y) for y in ys], [20.0, 20.0], p)
    for y, o in zip(ys, outs):
        assert torch.equal(o, api.hts_denoise(T(y), 20.0, p))


def test_backward_rejects_the_flag():
    y = synth.tiny(804, 3, 32, 32, sigma=15.0)
    p = api.Params(stride=3, window=9, K=8, flags=FT)
    out, st = api.hts_denoise(T(y), 15.0, p, save=True)
    with pytest.raises(api.L.HtsError):
        api.hts_denoise_backward(torch.ones_like(out), st, p)
