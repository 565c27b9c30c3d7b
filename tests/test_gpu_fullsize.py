"""Parity at full size, in the launch configuration bench.py times: the
64-image mixed-size RGB batch through hts_denoise_batch (s3 w31 K32, the
autotuned schedule), checked against the FP64 oracle on samples it can
compute one by one:
  * sampled references of three images (the largest, a middle and a small
    one): the exact top-K of the brute-force window scan;
  * the FP64 basis of those images;
  * sampled output pixels: every group with a patch over the pixel is
    filtered by the oracle (Eq. 18-20 under the GPU's keep-masks, the
    threshold-kink protocol of the small tests, GPU float basis) and
    averaged (Eq. 2); the pixel must agree within 1e-3.
The batch output of each image equals its single-image hts_denoise bit for
bit (the bench's timed path is the batched one).  The same checks on the
4000 x 6000 RGB image (stride 2, window 39), on one 520 x 696 x 34
spectral-tube image through the band-count path and on an
eight-frame 540 x 960 RGB video; the gradient of the differentiable
configuration at sampled pixels."""
import concurrent.futures
import multiprocessing

import numpy as np
import pytest
import torch

from oracle import basis as obasis
from oracle import filtering as of
from oracle import matching as omatch
from oracle.grid import ref_grid
from paper_2508_10307_amd import api, synth

pytestmark = pytest.mark.gpu

PIX_TOL = 1e-3
DELTA_REL = 2e-4


def dev():
    return torch.device("cuda:0")


def log(*a):
    print(*a, flush=True)


def group_masks(words, g, K, C):
    """Keep-masks of group g from the bit-packed stream, bool [K, C, 8, 8]."""
    n = K * C * 2
    w = np.ascontiguousarray(words[g * n:(g + 1) * n], dtype="<u4")
    bits = np.unpackbits(w.view(np.uint8), bitorder="little")
    return bits.astype(bool).reshape(K, C, 8, 8)


@pytest.fixture(scope="module")
def batch():
    wl = synth.batch64()
    q = wl.params
    xs = [torch.from_numpy(im.noisy).to(dev()) for im in wl.images]
    # the schedule bench.py picks: the autotuner on the largest image shape
    th, tw = max(x.shape[1] for x in xs), max(x.shape[2] for x in xs)
    tune = api.hts_autotune(api.Params(stride=q.stride, window=q.window, K=q.K,
                                       tau_mult=q.tau_mult), 3, th, tw)
    log("autotuned schedule", tune)
    p = api.Params(stride=q.stride, window=q.window, K=q.K, tau_mult=q.tau_mult, tune=tune)
    sig = [im.sigma for im in wl.images]
    outs = api.hts_denoise_batch(xs, sig, p)
    torch.cuda.synchronize()
    return wl, p, xs, sig, outs


def picks(wl):
    """Six images: the largest, the smallest, a middle one, and the most
    elongated ones (W / H largest and smallest), plus the one with the
    highest noise level."""
    areas = [im.noisy.shape[1] * im.noisy.shape[2] for im in wl.images]
    order = np.argsort(areas, kind="stable")
    aspect = np.argsort([im.noisy.shape[2] / im.noisy.shape[1] for im in wl.images], kind="stable")
    noisiest = int(np.argmax([im.sigma for im in wl.images]))
    out = []
    for i in (order[-1], order[0], order[len(order) // 2], aspect[-1], aspect[0], noisiest):
        if int(i) not in out:
            out.append(int(i))
    return out


def test_fullsize_batch_samples_match_the_oracle(batch):
    wl, p, xs, sig, outs = batch
    rng = np.random.default_rng(11)
    K, s, w = p.K, p.stride, p.window
    r = (w - 1) // 2
    for i in picks(wl):
        y = wl.images[i].noisy
        C, H, W = y.shape
        log(f"image {i}: {H}x{W}, sigma {sig[i]:.2f}")
        out1, st = api.hts_denoise(xs[i], sig[i], p, save=True)
        assert torch.equal(out1, outs[i])
        idx = st["idx"].cpu().numpy().astype(np.int64)
        words = st["masks"].cpu().numpy().view(np.uint32)
        # sampled references: brute-force window scan
        ys, xs_, _, _ = ref_grid(H, W, 8, s)
        qg = omatch.quantize(y)
        planes = omatch.guide_planes(qg)
        green = omatch.gcp_green(qg, ys, xs_, 8, p.gcp_num, p.gcp_den)
        Hp, Wp = H - 7, W - 7
        for n in rng.choice(len(ys), 60, replace=False):
            ry, rx = int(ys[n]), int(xs_[n])
            pl = planes[0 if green[n] else 1]
            ref = pl[ry:ry + 8, rx:rx + 8]
            c = []
            for cy in range(max(0, ry - r), min(Hp - 1, ry + r) + 1):
                for cx in range(max(0, rx - r), min(Wp - 1, rx + r) + 1):
                    if (cy, cx) != (ry, rx):
                        c.append((int(((pl[cy:cy + 8, cx:cx + 8] - ref) ** 2).sum()), cy * W + cx))
            c.sort()
            assert list(idx[n]) == [ry * W + rx] + [v for _, v in c[:K - 1]], (i, n)
        # FP64 basis
        _, _, U64, V64, _ = api.hts_basis(xs[i], p, want_fp64=True)
        _, _, Uo, Vo, _, _ = obasis.global_basis(y.astype(np.float64), 8, s)
        np.testing.assert_allclose(U64.cpu().numpy(), Uo, atol=1e-9)
        np.testing.assert_allclose(V64.cpu().numpy(), Vo, atol=1e-9)
        # sampled output pixels
        UF = obasis.fourier_from_real(st["U"].cpu().numpy().astype(np.float64))
        VF = obasis.fourier_from_real(st["V"].cpu().numpy().astype(np.float64))
        tau = p.tau_mult * sig[i]
        py, px = np.divmod(idx, W)
        out = outs[i].cpu().numpy()
        for _ in range(6):
            yy, xx = int(rng.integers(0, H)), int(rng.integers(0, W))
            cover = (py <= yy) & (yy < py + 8) & (px <= xx) & (xx < px + 8)
            gs = np.nonzero(cover.any(axis=1))[0]
            G = of.gather_groups(y.astype(np.float64), idx[gs], 8)
            S = of.haar_group(of.tsvd_forward(G, UF, VF), K)
            M = np.stack([group_masks(words, int(g), K, C) for g in gs])
            keep = np.abs(S) >= tau
            diff = M != keep
            if diff.any():
                assert np.abs(np.abs(S[diff]) - tau).max() <= DELTA_REL * max(tau, 1.0)
            est = of.tsvd_inverse(of.haar_group_inverse(np.where(M, S, 0.0), K), UF, VF)
            num = np.zeros(C)
            cnt = 0
            for gi, g in enumerate(gs):
                for k in np.nonzero(cover[g])[0]:
                    num += est[gi, k, :, yy - py[g, k], xx - px[g, k]]
                    cnt += 1
            err = np.abs(out[:, yy, xx] - num / cnt).max()
            log(f"  pixel ({yy},{xx}): {len(gs)} groups, {cnt} estimates, |gpu - oracle| = {err:.2e}")
            assert err <= PIX_TOL


def _covariance_part(args):
    """The oracle's per-frequency covariances over references [b0, b1) of
    the image saved at path (a worker process of the large-image test)."""
    path, s, b0, b1 = args
    y = np.load(path, mmap_mode="r")
    C, H, W = y.shape
    ys, xs_, _, _ = ref_grid(H, W, 8, s)
    a = np.arange(8)
    CU = CV = None
    for c0 in range(b0, b1, 100000):
        c1 = min(b1, c0 + 100000)
        yy_, xx_ = ys[c0:c1], xs_[c0:c1]
        P = np.asarray(y)[:, yy_[:, None, None] + a[None, :, None],
                          xx_[:, None, None] + a[None, None, :]]
        cu, cv = obasis.covariances(np.ascontiguousarray(np.moveaxis(P, 0, 1)))
        CU = cu if CU is None else [u + v for u, v in zip(CU, cu)]
        CV = cv if CV is None else [u + v for u, v in zip(CV, cv)]
    return CU, CV


def test_fullsize_large_image_samples_match_the_oracle(tmp_path):
    """The 24 MPix configuration (RGB 4000 x 6000, 400 blobs, AWGN sigma = 15,
    stride 2, window 39, K 32; 5,985,009 references, 766 MB of indices),
    through hts_denoise as bench.py's large_image object runs it: sampled
    references against the brute-force window scan (among them the last
    reference rows and columns and the corners), BF16 and FP32 matching
    equal over the whole index array, the FP64 basis against the oracle's
    covariances summed over every reference patch (in chunks), and sampled
    output pixels recomputed from every group over them."""
    wl = synth.large_24mpix()
    im, q = wl.images[0], wl.params
    y = im.noisy
    C, H, W = y.shape
    K, s, w = q.K, q.stride, q.window
    r = (w - 1) // 2
    p = api.Params(stride=s, window=w, K=K, tau_mult=q.tau_mult)
    x = torch.from_numpy(y).to(dev())
    out, st = api.hts_denoise(x, im.sigma, p, save=True)
    torch.cuda.synchronize()
    idx_t = st["idx"]
    n_ref = idx_t.shape[0]
    log(f"large image: {H}x{W}, {n_ref} references")
    assert n_ref == 5985009
    i32 = api.hts_match(x, api.Params(stride=s, window=w, K=K, match_mode=1))
    assert torch.equal(i32, idx_t)
    del i32
    # sampled references, brute force
    ys, xs_, ny, nx = ref_grid(H, W, 8, s)
    qg = omatch.quantize(y)
    planes = omatch.guide_planes(qg)
    Hp, Wp = H - 7, W - 7
    rng = np.random.default_rng(24)
    sample = list(rng.choice(n_ref, 30, replace=False)) + [0, nx - 1, n_ref - nx, n_ref - 1,
                                                           (ny // 2) * nx + nx - 1]
    rows = idx_t[torch.tensor(sample, device=dev())].cpu().numpy().astype(np.int64)
    green = omatch.gcp_green(qg, ys[sample], xs_[sample], 8, p.gcp_num, p.gcp_den)
    for j, n in enumerate(sample):
        ry, rx = int(ys[n]), int(xs_[n])
        pl = planes[0 if green[j] else 1]
        ref = pl[ry:ry + 8, rx:rx + 8]
        c = []
        for cy in range(max(0, ry - r), min(Hp - 1, ry + r) + 1):
            for cx in range(max(0, rx - r), min(Wp - 1, rx + r) + 1):
                if (cy, cx) != (ry, rx):
                    c.append((int(((pl[cy:cy + 8, cx:cx + 8] - ref) ** 2).sum()), cy * W + cx))
        c.sort()
        assert list(rows[j]) == [ry * W + rx] + [v for _, v in c[:K - 1]], n
    log("  sampled references exact")
    # FP64 basis: the oracle's covariances of all 6M reference patches, in
    # 16 CPU worker processes (chunks of the reference list, summed in order)
    y64 = y.astype(np.float64)
    np.save(tmp_path / "y.npy", y64)
    bounds = np.linspace(0, n_ref, 17).astype(int)
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(16, mp_context=ctx) as ex:
        parts = list(ex.map(_covariance_part, [(str(tmp_path / "y.npy"), s, int(b0), int(b1))
                                               for b0, b1 in zip(bounds[:-1], bounds[1:])]))
    CU = [sum(pt[0][f] for pt in parts) for f in range(C // 2 + 1)]
    CV = [sum(pt[1][f] for pt in parts) for f in range(C // 2 + 1)]
    _, _, Uo, Vo, _, _ = obasis.basis_from_covariances(CU, CV, C)
    _, _, U64, V64, _ = api.hts_basis(x, p, want_fp64=True)
    np.testing.assert_allclose(U64.cpu().numpy(), Uo, atol=1e-9)
    np.testing.assert_allclose(V64.cpu().numpy(), Vo, atol=1e-9)
    log("  FP64 basis within 1e-9")
    # sampled output pixels (groups found on the device)
    UF = obasis.fourier_from_real(st["U"].cpu().numpy().astype(np.float64))
    VF = obasis.fourier_from_real(st["V"].cpu().numpy().astype(np.float64))
    tau = q.tau_mult * im.sigma
    py_t, px_t = idx_t // W, idx_t % W
    nw = K * C * 2
    for yy, xx in [(int(rng.integers(0, H)), int(rng.integers(0, W))) for _ in range(2)] + \
            [(H - 1, W - 1), (0, 0)]:
        cov_t = (py_t <= yy) & (yy < py_t + 8) & (px_t <= xx) & (xx < px_t + 8)
        gs_t = torch.nonzero(cov_t.any(dim=1)).flatten()
        gs = gs_t.cpu().numpy()
        gidx = idx_t[gs_t].cpu().numpy().astype(np.int64)
        wsel = (gs_t[:, None] * nw + torch.arange(nw, device=dev())[None]).flatten()
        words = st["masks"][wsel].cpu().numpy().view(np.uint32)
        gpy, gpx = np.divmod(gidx, W)
        cover = (gpy <= yy) & (yy < gpy + 8) & (gpx <= xx) & (xx < gpx + 8)
        S = of.haar_group(of.tsvd_forward(of.gather_groups(y64, gidx, 8), UF, VF), K)
        M = np.stack([group_masks(words, gi, K, C) for gi in range(len(gs))])
        diff = M != (np.abs(S) >= tau)
        if diff.any():
            assert np.abs(np.abs(S[diff]) - tau).max() <= DELTA_REL * tau
        est = of.tsvd_inverse(of.haar_group_inverse(np.where(M, S, 0.0), K), UF, VF)
        num, cnt = np.zeros(C), 0
        for gi in range(len(gs)):
            for k in np.nonzero(cover[gi])[0]:
                num += est[gi, k, :, yy - gpy[gi, k], xx - gpx[gi, k]]
                cnt += 1
        o = out[:, yy, xx].cpu().numpy()
        err = np.abs(o - num / cnt).max()
        log(f"  pixel ({yy},{xx}): {len(gs)} groups, {cnt} estimates, |gpu - oracle| = {err:.2e}")
        assert err <= PIX_TOL


def test_fullsize_spectral_tube_samples_match_the_oracle():
    """One 520 x 696 x 34 image (the size of the paper's real-HSI scenes)
    through the band-count path, as bench.py's spectral_tubes object runs
    it: sampled references, the FP64 basis and sampled output pixels."""
    C, H, W = 34, 520, 696
    clean = synth.clean_image(4242, 0, C, H, W, 40)
    y = synth.add_awgn(4242, 0, clean, 25.0)
    p = api.Params(stride=3, window=31, K=32)
    x = torch.from_numpy(y).to(dev())
    out, st = api.hts_denoise(x, 25.0, p, save=True)
    idx = st["idx"].cpu().numpy().astype(np.int64)
    words = st["masks"].cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(12)
    K, s, r = p.K, p.stride, (p.window - 1) // 2
    ys, xs_, _, _ = ref_grid(H, W, 8, s)
    g = omatch.guide_planes(omatch.quantize(y))[0]
    Hp, Wp = H - 7, W - 7
    for n in rng.choice(len(ys), 20, replace=False):
        ry, rx = int(ys[n]), int(xs_[n])
        ref = g[ry:ry + 8, rx:rx + 8]
        c = []
        for cy in range(max(0, ry - r), min(Hp - 1, ry + r) + 1):
            for cx in range(max(0, rx - r), min(Wp - 1, rx + r) + 1):
                if (cy, cx) != (ry, rx):
                    c.append((int(((g[cy:cy + 8, cx:cx + 8] - ref) ** 2).sum()), cy * W + cx))
        c.sort()
        assert list(idx[n]) == [ry * W + rx] + [v for _, v in c[:K - 1]], n
    _, _, U64, V64, _ = api.hts_basis(x, p, want_fp64=True)
    _, _, Uo, Vo, _, _ = obasis.global_basis(y.astype(np.float64), 8, s)
    np.testing.assert_allclose(U64.cpu().numpy(), Uo, atol=1e-9)
    np.testing.assert_allclose(V64.cpu().numpy(), Vo, atol=1e-9)
    UF = obasis.fourier_from_real(st["U"].cpu().numpy().astype(np.float64))
    VF = obasis.fourier_from_real(st["V"].cpu().numpy().astype(np.float64))
    tau = p.tau_mult * 25.0
    py, px = np.divmod(idx, W)
    o = out.cpu().numpy()
    for _ in range(3):
        yy, xx = int(rng.integers(0, H)), int(rng.integers(0, W))
        cover = (py <= yy) & (yy < py + 8) & (px <= xx) & (xx < px + 8)
        gs = np.nonzero(cover.any(axis=1))[0]
        S = of.haar_group(of.tsvd_forward(of.gather_groups(y.astype(np.float64), idx[gs], 8),
                                          UF, VF), K)
        M = np.stack([group_masks(words, int(q), K, C) for q in gs])
        diff = M != (np.abs(S) >= tau)
        if diff.any():
            assert np.abs(np.abs(S[diff]) - tau).max() <= DELTA_REL * tau
        est = of.tsvd_inverse(of.haar_group_inverse(np.where(M, S, 0.0), K), UF, VF)
        num, cnt = np.zeros(C), 0
        for gi, q in enumerate(gs):
            for k in np.nonzero(cover[q])[0]:
                num += est[gi, k, :, yy - py[q, k], xx - px[q, k]]
                cnt += 1
        err = np.abs(o[:, yy, xx] - num / cnt).max()
        log(f"  tube pixel ({yy},{xx}): {len(gs)} groups, |gpu - oracle| = {err:.2e}")
        assert err <= PIX_TOL


def test_fullsize_adjoint_samples_match_the_oracle():
    """The differentiable configuration (512 x 512 RGB, K = 16, w = 31, loss =
    mean squared error to the clean image): autograd through HaarTSVD, the
    input gradient checked at sampled pixels against the oracle's frozen
    adjoint (every group over the pixel, its K patches of g / cnt through
    Q^T M Q with the forward masks)."""
    wl = synth.diff_batch16(n=1)
    im, q = wl.images[0], wl.params
    p = api.Params(stride=q.stride, window=q.window, K=q.K, tau_mult=q.tau_mult)
    x = torch.from_numpy(im.noisy).to(dev()).requires_grad_(True)
    clean = torch.from_numpy(im.clean.astype(np.float32)).to(dev())
    out = api.HaarTSVD.apply(x, im.sigma, q.tau_mult, p)
    ((out - clean) ** 2).mean().backward()
    g = (2.0 * (out.detach() - clean) / out.numel()).cpu().numpy().astype(np.float64)
    _, st = api.hts_denoise(x.detach(), im.sigma, p, save=True)
    C, H, W = im.noisy.shape
    K = q.K
    idx = st["idx"].cpu().numpy().astype(np.int64)
    words = st["masks"].cpu().numpy().view(np.uint32)
    r = g / st["cnt"].cpu().numpy().astype(np.float64)[None]
    UF = obasis.fourier_from_real(st["U"].cpu().numpy().astype(np.float64))
    VF = obasis.fourier_from_real(st["V"].cpu().numpy().astype(np.float64))
    py, px = np.divmod(idx, W)
    grad = x.grad.cpu().numpy()
    scale = np.abs(grad).max()
    rng = np.random.default_rng(13)
    for _ in range(4):
        yy, xx = int(rng.integers(0, H)), int(rng.integers(0, W))
        cover = (py <= yy) & (yy < py + 8) & (px <= xx) & (xx < px + 8)
        gs = np.nonzero(cover.any(axis=1))[0]
        S = of.haar_group(of.tsvd_forward(of.gather_groups(r, idx[gs], 8), UF, VF), K)
        M = np.stack([group_masks(words, int(q_), K, C) for q_ in gs])
        est = of.tsvd_inverse(of.haar_group_inverse(np.where(M, S, 0.0), K), UF, VF)
        acc = np.zeros(C)
        for gi, q_ in enumerate(gs):
            for k in np.nonzero(cover[q_])[0]:
                acc += est[gi, k, :, yy - py[q_, k], xx - px[q_, k]]
        err = np.abs(grad[:, yy, xx] - acc).max()
        log(f"  gradient at ({yy},{xx}): {len(gs)} groups, |gpu - oracle| = {err:.2e} (max |grad| {scale:.2e})")
        assert err <= 1e-4 * scale


def test_fullsize_video_samples_match_the_oracle():
    """Eight 540 x 960 RGB frames with temporal reach 2 (bench.py's video
    object): sampled references against the brute-force spatio-temporal
    scan, the sequence basis in float, and sampled output pixels recomputed
    from every group over them (stacked coordinates)."""
    from oracle import video as ovideo
    Tn, C, H, W, dt = 8, 3, 540, 960, 2
    clean = synth.clean_video(4343, Tn, C, H, W, 40)
    f = np.stack([synth.add_awgn(4343, t, clean[t], 25.0) for t in range(Tn)])
    p = api.Params(stride=3, window=21, K=32)
    x = torch.from_numpy(f).to(dev())
    out, st = api.hts_denoise_video(x, 25.0, p, dt=dt, save=True)
    idx = st["idx"].cpu().numpy().astype(np.int64)
    words = st["masks"].cpu().numpy().view(np.uint32)
    K, s, r = p.K, p.stride, (p.window - 1) // 2
    ys, xs_, _, _ = ref_grid(H, W, 8, s)
    n_f = len(ys)
    q = [omatch.quantize(f[t]) for t in range(Tn)]
    planes = [omatch.guide_planes(qq) for qq in q]
    rng = np.random.default_rng(14)
    Hp, Wp = H - 7, W - 7
    for ref in rng.choice(Tn * n_f, 12, replace=False):
        t, n = divmod(int(ref), n_f)
        ry, rx = int(ys[n]), int(xs_[n])
        green = omatch.gcp_green(q[t], ys[n:n + 1], xs_[n:n + 1], 8, p.gcp_num, p.gcp_den)[0]
        pl = 0 if green else 1
        refp = planes[t][pl][ry:ry + 8, rx:rx + 8]
        c = []
        for t2 in range(max(0, t - dt), min(Tn - 1, t + dt) + 1):
            gp = planes[t2][pl]
            for cy in range(max(0, ry - r), min(Hp - 1, ry + r) + 1):
                for cx in range(max(0, rx - r), min(Wp - 1, rx + r) + 1):
                    if (t2, cy, cx) != (t, ry, rx):
                        c.append((int(((gp[cy:cy + 8, cx:cx + 8] - refp) ** 2).sum()),
                                  (t2 * H + cy) * W + cx))
        c.sort()
        assert list(idx[ref]) == [(t * H + ry) * W + rx] + [v for _, v in c[:K - 1]], ref
    _, _, Uo, Vo, _, _ = ovideo.global_basis(f.astype(np.float64), 8, s)
    np.testing.assert_allclose(st["U"].cpu().numpy(), Uo, atol=2e-6)
    np.testing.assert_allclose(st["V"].cpu().numpy(), Vo, atol=2e-6)
    UF = obasis.fourier_from_real(st["U"].cpu().numpy().astype(np.float64))
    VF = obasis.fourier_from_real(st["V"].cpu().numpy().astype(np.float64))
    ystack = ovideo.stack(f.astype(np.float64))
    ostack = ovideo.stack(out.cpu().numpy())
    tau = p.tau_mult * 25.0
    py, px = np.divmod(idx, W)
    for _ in range(3):
        yy, xx = int(rng.integers(0, Tn * H)), int(rng.integers(0, W))
        cover = (py <= yy) & (yy < py + 8) & (px <= xx) & (xx < px + 8)
        gs = np.nonzero(cover.any(axis=1))[0]
        S = of.haar_group(of.tsvd_forward(of.gather_groups(ystack, idx[gs], 8), UF, VF), K)
        M = np.stack([group_masks(words, int(q_), K, C) for q_ in gs])
        diff = M != (np.abs(S) >= tau)
        if diff.any():
            assert np.abs(np.abs(S[diff]) - tau).max() <= DELTA_REL * tau
        est = of.tsvd_inverse(of.haar_group_inverse(np.where(M, S, 0.0), K), UF, VF)
        num, cnt = np.zeros(C), 0
        for gi, q_ in enumerate(gs):
            for k in np.nonzero(cover[q_])[0]:
                num += est[gi, k, :, yy - py[q_, k], xx - px[q_, k]]
                cnt += 1
        err = np.abs(ostack[:, yy, xx] - num / cnt).max()
        log(f"  video pixel (row {yy}, col {xx}): {len(gs)} groups, |gpu - oracle| = {err:.2e}")
        assert err <= PIX_TOL
