"""GPU parity of the general band counts (spectral tubes, reading H1) with the
FP64 oracle, through the C ABI: match indices bit-exact (band-mean guide),
the FP64 basis within 1e-9, and the denoised image within 1e-3 on the
0..255 scale under the GPU's exported keep-masks (the threshold-kink
protocol of the RGB tests); equal bands reproduce the grey result, a NaN
band pixel makes the whole output NaN, and repeated calls give the same
bits."""
import numpy as np
import pytest
import torch

from oracle import basis as obasis
from oracle import matching as om
from oracle import pipeline as opipe
from paper_2508_10307_amd import api, synth

pytestmark = pytest.mark.gpu

PIX_TOL = 1e-3
DELTA_REL = 2e-4
CASES = [(2, 32, 30, 3, 9, 8), (5, 36, 33, 3, 11, 16), (8, 29, 28, 2, 11, 32),
         (31, 24, 26, 3, 9, 8), (4, 27, 25, 3, 9, 2)]


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev())


def log(*a):
    print(*a, flush=True)


def tube(C, H, W, seed, sigma=20.0):
    return synth.tiny(seed, C, H, W, sigma=sigma, n_blobs=5)


@pytest.mark.parametrize("C,H,W,s,w,K", CASES)
def test_match_and_basis_match_oracle(C, H, W, s, w, K):
    y = tube(C, H, W, 2100 + C)
    p = api.Params(stride=s, window=w, K=K)
    x = T(y)
    idx = api.hts_match(x, p)
    idx_o, _, _ = om.match(y, 8, s, w, K)
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), idx_o)
    U, V, U64, V64, eig = api.hts_basis(x, p, want_fp64=True)
    _, _, Uo, Vo, eUo, eVo = obasis.global_basis(y.astype(np.float64), 8, s)
    np.testing.assert_allclose(U64.cpu().numpy(), Uo, atol=1e-9)
    np.testing.assert_allclose(V64.cpu().numpy(), Vo, atol=1e-9)
    ev = eig.cpu().numpy()
    np.testing.assert_allclose(ev[0], eUo, rtol=1e-11, atol=1e-9 * eUo.max())
    np.testing.assert_allclose(ev[1], eVo, rtol=1e-11, atol=1e-9 * eVo.max())


@pytest.mark.parametrize("C,H,W,s,w,K", CASES)
def test_denoise_matches_oracle(C, H, W, s, w, K):
    sigma = 20.0
    y = tube(C, H, W, 2200 + C, sigma)
    p = api.Params(stride=s, window=w, K=K)
    x = T(y)
    out, st = api.hts_denoise(x, sigma, p, save=True)
    out2 = api.hts_denoise(x, sigma, p)
    assert torch.equal(out, out2)
    idx = st["idx"].cpu().numpy().astype(np.int64)
    masks = opipe.unpack_masks(st["masks"].cpu().numpy().view(np.uint32), len(idx), K, C)
    r = opipe.denoise(y, sigma, 8, s, w, K, p.tau_mult, idx=idx, U=st["U"].cpu().numpy(),
                      V=st["V"].cpu().numpy(), mask=masks)
    tau = p.tau_mult * sigma
    log(f"C{C}: overrides {r['n_override']}, max margin {r['max_override_margin']:.3e}")
    assert r["max_override_margin"] <= DELTA_REL * max(tau, 1.0)
    err = np.abs(out.cpu().numpy() - r["out"]).max()
    log(f"C{C} {H}x{W} s{s} w{w} K{K}: max |gpu - oracle| = {err:.3e}")
    assert err <= PIX_TOL
    np.testing.assert_array_equal(st["cnt"].cpu().numpy(), r["cnt"])


def test_equal_bands_give_the_grey_result():
    g = synth.tiny(2301, 1, 36, 34, sigma=20.0)
    p = api.Params(stride=3, window=11, K=16)
    grey = api.hts_denoise(T(g), 20.0, p)
    tubes = api.hts_denoise(T(np.repeat(g, 4, axis=0)), 20.0, p)
    for ch in range(4):
        assert (tubes[ch] - grey[0]).abs().max().item() <= PIX_TOL


def test_zero_sigma_reconstructs():
    y = tube(6, 30, 31, 2302)
    out = api.hts_denoise(T(y), 0.0, api.Params(stride=3, window=9, K=8))
    assert (out - T(y)).abs().max().item() <= 1e-3


def test_nan_band_pixel_makes_the_output_nan():
    y = tube(5, 30, 28, 2303, 10.0)
    y[3, 11, 7] = np.nan
    out = api.hts_denoise(T(y), 10.0, api.Params(stride=3, window=9, K=8))
    assert torch.isnan(out).all()


@pytest.mark.parametrize("C,K,s", [(256, 4, 3), (2, 32, 1), (12, 2, 8)])
def test_band_count_extremes(C, K, s):
    """The largest band count, stride 1 with the largest group, stride 8 with
    the smallest group: the same parity bar."""
    sigma = 15.0
    H, W, w = 20, 22, 11
    y = tube(C, H, W, 2400 + C + K, sigma)
    p = api.Params(stride=s, window=w, K=K)
    x = T(y)
    out, st = api.hts_denoise(x, sigma, p, save=True)
    idx = st["idx"].cpu().numpy().astype(np.int64)
    idx_o, _, _ = om.match(y, 8, s, w, K)
    np.testing.assert_array_equal(idx, idx_o)
    masks = opipe.unpack_masks(st["masks"].cpu().numpy().view(np.uint32), len(idx), K, C)
    r = opipe.denoise(y, sigma, 8, s, w, K, p.tau_mult, idx=idx, U=st["U"].cpu().numpy(),
                      V=st["V"].cpu().numpy(), mask=masks)
    assert r["max_override_margin"] <= DELTA_REL * max(p.tau_mult * sigma, 1.0)
    err = np.abs(out.cpu().numpy() - r["out"]).max()
    log(f"C{C} K{K} s{s}: max |gpu - oracle| = {err:.3e}, overrides {r['n_override']}")
    assert err <= PIX_TOL


def test_band_count_entry_points_refuse_unbuilt_calls():
    y = tube(5, 24, 24, 2500)
    x = T(y)
    p = api.Params(stride=3, window=9, K=8)
    _, st = api.hts_denoise(x, 10.0, p, save=True)
    with pytest.raises(api.L.HtsError):
        api.hts_denoise_batch([x], [10.0], p)
    with pytest.raises(api.L.HtsError):
        api.hts_denoise(x, 10.0, api.Params(stride=3, window=9, K=8, flags=api.L.HTS_FLAG_WEIGHTED))


def test_filter_entry_point_for_band_counts():
    """hts_filter over two reference ranges adds the same numerator and
    counts as hts_denoise forms (float atomics: within 1e-3 after the
    division); its per-group estimates equal the oracle's for the GPU's
    masks and basis."""
    C, H, W, s, w, K = 6, 30, 28, 3, 9, 8
    sigma = 18.0
    y = tube(C, H, W, 2600, sigma)
    p = api.Params(stride=s, window=w, K=K)
    x = T(y)
    out, st = api.hts_denoise(x, sigma, p, save=True)
    n_ref = st["idx"].shape[0]
    half = n_ref // 2
    a = api.hts_filter(x, sigma, st["idx"], st["U"], st["V"], p, 0, half, want_group_est=True,
                       want_masks=True)
    b = api.hts_filter(x, sigma, st["idx"], st["U"], st["V"], p, half, n_ref - half)
    num = (a["num"] + b["num"]).cpu().numpy()
    cnt = (a["cnt"] + b["cnt"]).cpu().numpy()
    np.testing.assert_array_equal(cnt, st["cnt"].cpu().numpy())
    assert np.abs(num / cnt[None] - out.cpu().numpy()).max() <= PIX_TOL
    idx = st["idx"].cpu().numpy().astype(np.int64)
    masks = opipe.unpack_masks(a["masks"].cpu().numpy().view(np.uint32), half, K, C)
    from oracle import basis as ob, filtering as of
    UF = ob.fourier_from_real(st["U"].cpu().numpy().astype(np.float64))
    VF = ob.fourier_from_real(st["V"].cpu().numpy().astype(np.float64))
    S = of.haar_group(of.tsvd_forward(of.gather_groups(y.astype(np.float64), idx[:half], 8),
                                      UF, VF), K)
    est = of.tsvd_inverse(of.haar_group_inverse(np.where(masks, S, 0.0), K), UF, VF)
    err = np.abs(a["group_est"].cpu().numpy() - est).max()
    log(f"group estimates: max |gpu - oracle| = {err:.3e}")
    assert err <= PIX_TOL


@pytest.mark.parametrize("C,K", [(5, 8), (2, 16)])
def test_adjoint_for_band_counts_matches_oracle(C, K):
    """hts_denoise_backward with band counts other than 1 and 3: the
    transpose of the frozen-mask map against the oracle's frozen adjoint."""
    from oracle import adjoint as oadj
    H, W, s, w = 30, 29, 3, 11
    y = tube(C, H, W, 2700 + C, 15.0)
    p = api.Params(stride=s, window=w, K=K)
    x = T(y)
    _, st = api.hts_denoise(x, 15.0, p, save=True)
    g = np.random.default_rng(C).normal(size=y.shape)
    gin, gtau = api.hts_denoise_backward(T(g), st, p)
    idx = st["idx"].cpu().numpy().astype(np.int64)
    masks = opipe.unpack_masks(st["masks"].cpu().numpy().view(np.uint32), len(idx), K, C)
    ref = oadj.frozen_adjoint(g, idx, masks, st["U"].cpu().numpy().astype(np.float64),
                              st["V"].cpu().numpy().astype(np.float64),
                              st["cnt"].cpu().numpy().astype(np.float64), K)
    err = np.abs(gin.cpu().numpy() - ref).max()
    log(f"C{C} K{K} adjoint: max |gpu - oracle| = {err:.3e}, max |oracle| = {np.abs(ref).max():.3e}")
    assert err <= 1e-4 * max(1.0, np.abs(ref).max())
    assert gtau.item() == 0.0
