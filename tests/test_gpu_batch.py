"""Batched persistent, graph-captured pipeline (hts_denoise_batch) and the
launch-schedule autotuner, through the C ABI.

Every image of a batch is independent (its own reference grid, basis and
sigma), so a batch must give, per image, the result of hts_denoise: the
same stages on the same data, with the estimates summed in fixed point, so
the outputs are equal bit for bit.
Graph replays are checked one by one against eager results, with other
GPU work and synchronisations in between.
"""
import os

import numpy as np
import pytest
import torch

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


SHAPES = [(3, 64, 96), (3, 40, 33), (3, 128, 70), (3, 33, 128), (3, 96, 96)]


def make_batch(seed):
    imgs, sig = [], []
    for i, (C, H, W) in enumerate(SHAPES):
        s = 5.0 + 9.0 * ((seed + i) % 5)
        imgs.append(synth.tiny(seed * 100 + i, C, H, W, sigma=s, n_blobs=6))
        sig.append(s)
    return imgs, sig


def eager(imgs, sig, p):
    return [api.hts_denoise(T(y), s, p) for y, s in zip(imgs, sig)]


def test_batch_matches_per_image_and_oracle():
    p = api.Params(stride=3, window=15, K=16)
    imgs, sig = make_batch(1)
    xs = [T(y) for y in imgs]
    outs = api.hts_denoise_batch(xs, sig, p)
    torch.cuda.synchronize()
    ref = eager(imgs, sig, p)
    for i, (o, r) in enumerate(zip(outs, ref)):
        err = (o - r).abs().max().item()
        log("batch vs eager", i, SHAPES[i], err)
        assert torch.equal(o, r)
    # one image of the batch against the oracle (mask protocol as in the single-image tests)
    y, s = imgs[2], sig[2]
    o2, st = api.hts_denoise(T(y), s, p, save=True)
    idx = st["idx"].cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(idx, omatch.match(y, 8, p.stride, p.window, p.K)[0])
    masks = opipe.unpack_masks(st["masks"].cpu().numpy().view(np.uint32), len(idx), p.K, 3)
    r = opipe.denoise(y, s, 8, p.stride, p.window, p.K, p.tau_mult, idx=idx,
                      U=st["U"].cpu().numpy(), V=st["V"].cpu().numpy(), mask=masks)
    assert np.abs(outs[2].cpu().numpy() - r["out"]).max() <= 1e-3


@pytest.mark.parametrize("mode", [0, 1], ids=["bf16", "fp32"])
def test_graph_replays_with_new_inputs(mode):
    p = api.Params(stride=3, window=15, K=16, match_mode=mode)
    C_shapes = SHAPES
    xs0 = [torch.empty((C, H, W), device=dev()) for C, H, W in C_shapes]
    outs = [torch.empty_like(x) for x in xs0]
    ws = torch.empty(api.batch_workspace_size(p, xs0, outs, [10.0] * len(xs0)),
                     dtype=torch.uint8, device=dev())
    for rep in range(4):
        imgs, sig = make_batch(10 + rep)
        xs = [T(y) for y in imgs]          # new pointers every replay
        api.hts_denoise_batch(xs, sig, p, outs=outs, ws=ws)
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device=dev()).sum()
        torch.cuda.synchronize()
        ref = eager(imgs, sig, p)
        for i, (o, r) in enumerate(zip(outs, ref)):
            err = (o - r).abs().max().item()
            log("replay", rep, i, err, float(junk))
            assert torch.equal(o, r)


def test_batch_rejects_mixed_channels_and_bad_sigma():
    p = api.Params(stride=3, window=15, K=16)
    a = torch.zeros((3, 40, 40), device=dev())
    b = torch.zeros((1, 40, 40), device=dev())
    with pytest.raises(RuntimeError):
        api.hts_denoise_batch([a, b], [10.0, 10.0], p)
    with pytest.raises(RuntimeError):
        api.hts_denoise_batch([a], [float("nan")], p)


def test_autotune_picks_a_valid_schedule_and_caches(tmp_path):
    p = api.Params(stride=3, window=31, K=32)
    cache = str(tmp_path / "tune.txt")
    with open(cache, "w") as f:
        f.write("garbage line without separator\ngfx950 C=3 s=3 w=31 K=32 mode=0|0\n")
    w = api.hts_autotune(p, 3, 256, 256, cache_path=cache)
    log("tune word", w)
    assert 1 <= (w & 15) <= 9 and ((w >> 4) & 3) in (1, 2)
    assert any(l.strip().endswith(f"|{w}") for l in open(cache))
    assert api.hts_autotune(p, 3, 256, 256, cache_path=cache) == w
    # the tuned schedule gives the same indices and (to summation order) the same output
    y = synth.tiny(77, 3, 80, 72, sigma=20.0)
    a = api.hts_denoise(T(y), 20.0, api.Params(stride=3, window=31, K=32, tune=w))
    b = api.hts_denoise(T(y), 20.0, api.Params(stride=3, window=31, K=32, tune=1 | (2 << 4)))
    assert (a - b).abs().max().item() <= 1e-3
    ia = api.hts_match(T(y), api.Params(stride=3, window=31, K=32, tune=w))
    ib = api.hts_match(T(y), api.Params(stride=3, window=31, K=32, tune=1 | (1 << 4)))
    assert torch.equal(ia, ib)


def test_graph_follows_a_schedule_changed_by_the_autotuner(tmp_path):
    """tune = 0 takes the schedule from the autotune table; a batch call
    after hts_autotune (here fed from a cache file) changes that table, and
    the next tune = 0 call must run the new schedule, not replay the graph
    captured for the old one.  The image shapes, parameters and workspace
    stay the same across the three calls."""
    p = api.Params(stride=3, window=13, K=16)
    imgs, sig = make_batch(21)
    xs = [T(y) for y in imgs]
    outs = [torch.empty_like(x) for x in xs]
    ws = torch.empty(api.batch_workspace_size(p, xs, outs, sig), dtype=torch.uint8,
                     device=dev())
    api.hts_denoise_batch(xs, sig, p, outs=outs, ws=ws)       # default schedule, graph cached
    torch.cuda.synchronize()
    first = [o.clone() for o in outs]
    ref0 = eager(imgs, sig, p)
    for o, r in zip(first, ref0):
        assert torch.equal(o, r)
    # a cached schedule for exactly these parameters: vector-ALU filter, 2x2
    # reference tiles, BF16 hi/lo split (tune word (6 + 1) | 2 << 4 | 1 << 6)
    word = 7 | (2 << 4) | (1 << 6)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{arch} C=3 s=3 w=13 K=16 mode=0 flags=0|{word}\n")
    assert api.hts_autotune(p, 3, 96, 96, cache_path=str(cache)) == word
    api.hts_denoise_batch(xs, sig, p, outs=outs, ws=ws)       # tune = 0 again
    torch.cuda.synchronize()
    ref = eager(imgs, sig, api.Params(stride=3, window=13, K=16, tune=word))
    for i, (o, r) in enumerate(zip(outs, ref)):
        log("after autotune", i, SHAPES[i], (o - r).abs().max().item())
        assert torch.equal(o, r)


def test_staged_batch_equals_the_graph_and_times_its_stages():
    """hts_denoise_batch_staged: the same kernels launched one by one with
    timing events at the stage boundaries; the output equals the graph's bit
    for bit and every stage has a non-negative duration."""
    p = api.Params(stride=3, window=15, K=16)
    imgs, sig = make_batch(31)
    xs = [T(y) for y in imgs]
    ref = api.hts_denoise_batch(xs, sig, p)
    outs = [torch.empty_like(x) for x in xs]
    ws = torch.empty(api.batch_workspace_size(p, xs, outs, sig), dtype=torch.uint8,
                     device=dev())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
    api.hts_denoise_batch_staged(xs, sig, p, outs, ws, ev)
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert torch.equal(o, r)
    ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(6)]
    log("stage ms", dict(zip(api.BATCH_STAGES, ms)))
    assert all(m >= 0.0 for m in ms) and ms[1] > 0.0 and ms[4] > 0.0
    with pytest.raises(RuntimeError):
        api.hts_denoise_batch_staged(xs, sig, p, outs, ws, ev[:6])


# ------------------------------------------------- batched forward state and adjoint
def _state_equal(a, b):
    for k in ("idx", "masks", "U", "V", "cnt"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("tune", [1, 1 | (1 << 6)], ids=["mfma", "valu"])
def test_batch_save_writes_the_per_image_state(tune):
    """hts_denoise_batch_save: outputs and every image's idx, masks, U, V and
    cnt equal those of hts_denoise(save) on that image alone, bit for bit
    (the batch's mask buffers start all ones, so every word is written)."""
    p = api.Params(stride=3, window=15, K=16, tune=tune)
    imgs, sig = make_batch(41)
    xs = [T(y) for y in imgs]
    states = [api.new_state(p, *x.shape, dev()) for x in xs]
    for st in states:
        st["masks"].fill_(-1)
    outs, states = api.hts_denoise_batch_save(xs, sig, p, states=states)
    torch.cuda.synchronize()
    for i, (x, s) in enumerate(zip(xs, sig)):
        o, st = api.hts_denoise(x, s, p, save=True)
        log("batch save", i, SHAPES[i])
        assert torch.equal(outs[i], o)
        _state_equal(states[i], st)
    # the plain batch is unchanged beside it
    for o, r in zip(api.hts_denoise_batch(xs, sig, p), outs):
        assert torch.equal(o, r)


@pytest.mark.parametrize("tune", [1, 1 | (1 << 6)], ids=["mfma", "valu"])
def test_batch_backward_equals_per_image_adjoint(tune):
    """hts_denoise_batch_backward gives each image's hts_denoise_backward
    bit for bit, on graph replays with new gradients and swapped states,
    and with grad_in written over grad_out."""
    p = api.Params(stride=3, window=15, K=16, tune=tune)
    imgs, sig = make_batch(43)
    xs = [T(y) for y in imgs]
    _, states = api.hts_denoise_batch_save(xs, sig, p)
    imgs2, sig2 = make_batch(44)   # the same shapes, other images: other state buffers
    _, states2 = api.hts_denoise_batch_save([T(y) for y in imgs2], sig2, p)
    rng = np.random.default_rng(9)
    n = len(xs)
    ws = None
    for rep in range(3):
        gs = [T(rng.normal(size=x.shape)) for x in xs]
        sts = states2 if rep == 1 else states
        gins = [torch.empty_like(g) for g in gs]
        if ws is None:
            ws = torch.empty(api.batch_workspace_size(p, gs, gins, [0.0] * n), dtype=torch.uint8,
                             device=dev())
        api.hts_denoise_batch_backward(gs, sts, p, grad_ins=gins, ws=ws)
        torch.cuda.synchronize()
        for i in range(n):
            ref, gtau = api.hts_denoise_backward(gs[i], sts[i], p)
            assert torch.equal(gins[i], ref), (rep, i)
            assert gtau.item() == 0.0
        x2 = torch.randn(64, 64, device=dev())   # other GPU work between replays
        (x2 @ x2).sum().item()
    # in place: grad_in over grad_out
    gs = [T(rng.normal(size=x.shape)) for x in xs]
    refs = [api.hts_denoise_backward(g, st, p)[0] for g, st in zip(gs, states)]
    api.hts_denoise_batch_backward(gs, states, p, grad_ins=gs, ws=ws)
    torch.cuda.synchronize()
    for g, r in zip(gs, refs):
        assert torch.equal(g, r)


def test_batch_backward_adjoint_identity_and_oracle():
    """<D a, z> = <a, D^T z> for the frozen linear map D of every image
    (oracle frozen_forward), and one image's D^T z against the oracle's
    frozen adjoint."""
    from oracle import adjoint as oadj
    p = api.Params(stride=3, window=15, K=16)
    imgs, sig = make_batch(45)
    xs = [T(y) for y in imgs]
    _, states = api.hts_denoise_batch_save(xs, sig, p)
    rng = np.random.default_rng(11)
    zs = [rng.normal(size=y.shape) for y in imgs]
    gins = api.hts_denoise_batch_backward([T(z) for z in zs], states, p)
    torch.cuda.synchronize()
    for i in (0, 2, 4):
        st = states[i]
        idx = st["idx"].cpu().numpy().astype(np.int64)
        masks = opipe.unpack_masks(st["masks"].cpu().numpy().view(np.uint32), len(idx), p.K, 3)
        U, V, cnt = st["U"].cpu().numpy(), st["V"].cpu().numpy(), st["cnt"].cpu().numpy()
        a = rng.normal(size=imgs[i].shape)
        Da, cnt_o = oadj.frozen_forward(a, idx, masks, U, V, p.K)
        np.testing.assert_array_equal(cnt, cnt_o)
        gz = gins[i].cpu().numpy().astype(np.float64)
        lhs, rhs = np.vdot(Da, zs[i]), np.vdot(a, gz)
        log("batched adjoint dot", i, lhs, rhs)
        assert abs(lhs - rhs) <= 1e-4 * max(1.0, abs(lhs))
        ref = oadj.frozen_adjoint(zs[i], idx, masks, U, V, cnt_o, p.K)
        assert np.abs(gz - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("tune", [1, 1 | (1 << 6)], ids=["mfma", "valu"])
def test_batch_backward_takes_an_idx_from_a_larger_window(tune):
    """The batched adjoint accepts any grouping, as hts_denoise_backward
    does: groups of a window-25 match under window-9 parameters put patches
    outside the work group's tile (they go straight to the image)."""
    y = synth.tiny(4243, 3, 56, 60, sigma=20.0)
    x = T(y)
    _, st = api.hts_denoise(x, 20.0, api.Params(stride=3, window=25, K=16), save=True)
    pn = api.Params(stride=3, window=9, K=16, tune=tune)
    r = api.hts_filter(x, 20.0, st["idx"], st["U"], st["V"], pn, want_masks=True)
    st2 = dict(st, masks=r["masks"], cnt=r["cnt"])
    g = T(np.random.default_rng(6).normal(size=y.shape))
    ref, _ = api.hts_denoise_backward(g, st2, pn)
    y2 = synth.tiny(4244, 3, 40, 52, sigma=20.0)
    _, st3 = api.hts_denoise(T(y2), 20.0, pn, save=True)
    g2 = T(np.random.default_rng(7).normal(size=y2.shape))
    ref2, _ = api.hts_denoise_backward(g2, st3, pn)
    gins = api.hts_denoise_batch_backward([g, g2], [st2, st3], pn)
    torch.cuda.synchronize()
    assert torch.equal(gins[0], ref)
    assert torch.equal(gins[1], ref2)


def test_batch_save_and_backward_reject_bad_arguments():
    p = api.Params(stride=3, window=15, K=16)
    x = torch.zeros((3, 40, 40), device=dev())
    st = api.new_state(p, 3, 40, 40, dev())
    for flags in (1, 2):   # weighted aggregation, channel-Fourier threshold
        pf = api.Params(stride=3, window=15, K=16, flags=flags)
        with pytest.raises(RuntimeError):
            api.hts_denoise_batch_save([x], [10.0], pf, states=[st])
        with pytest.raises(RuntimeError):
            api.hts_denoise_batch_backward([x], [st], pf)
    bad = dict(st, cnt=torch.empty(0, device=dev()))   # data_ptr() of an empty tensor is null
    with pytest.raises(RuntimeError):
        api.hts_denoise_batch_backward([x], [bad], p)


def test_autograd_batch_equals_per_image_autograd():
    """HaarTSVDBatch over [N, C, H, W]: outputs and input gradients equal
    those of HaarTSVD image by image; the shared threshold multiplier's
    surrogate derivative is the sum of the images' derivatives, and the
    basis term adds in as per image."""
    p = api.Params(stride=3, window=15, K=16)
    N, C, H, W = 4, 3, 48, 56
    ys = [synth.tiny(700 + i, C, H, W, sigma=10.0 + 5 * i) for i in range(N)]
    sig = [10.0 + 5 * i for i in range(N)]
    clean = torch.stack([T(synth.tiny(700 + i, C, H, W, sigma=0.0)) for i in range(N)])
    for kappa, basis_grad in ((0.0, False), (0.1, True)):
        xb = torch.stack([T(y) for y in ys]).requires_grad_(True)
        tb = torch.tensor(2.7, device=dev(), requires_grad=True)
        ob = api.HaarTSVDBatch.apply(xb, sig, tb, p, kappa, basis_grad)
        ((ob - clean) ** 2).sum().backward()
        outs, grads, gt = [], [], []
        for i in range(N):
            xi = T(ys[i]).requires_grad_(True)
            ti = torch.tensor(2.7, device=dev(), requires_grad=True)
            oi = api.HaarTSVD.apply(xi, sig[i], ti, p, kappa, basis_grad)
            ((oi - clean[i]) ** 2).sum().backward()
            outs.append(oi.detach())
            grads.append(xi.grad)
            gt.append(ti.grad.item())
        torch.cuda.synchronize()
        assert torch.equal(ob.detach(), torch.stack(outs))
        assert torch.equal(xb.grad, torch.stack(grads))
        log("batched autograd", kappa, basis_grad, tb.grad.item(), sum(gt))
        if kappa == 0.0:
            assert tb.grad.item() == 0.0
        else:
            assert abs(tb.grad.item() - sum(gt)) <= 1e-5 * max(1.0, abs(sum(gt)))
    with pytest.raises(ValueError):
        api.HaarTSVDBatch.apply(xb.detach()[0], sig, 2.7, p)
    with pytest.raises(ValueError):
        api.HaarTSVDBatch.apply(xb.detach(), sig[:3], 2.7, p)


@pytest.mark.parametrize("K", [4, 16])
def test_batch_save_and_backward_gray(K):
    """Grey images (c = 1; K = 4 leaves slot lanes idle): the batched state
    export and the batched adjoint give the per-image bits."""
    p = api.Params(stride=2, window=11, K=K)
    shapes = [(1, 40, 52), (1, 33, 30), (1, 64, 48)]
    xs = [T(synth.tiny(800 + i, *sh, sigma=18.0)) for i, sh in enumerate(shapes)]
    sig = [18.0, 12.0, 25.0]
    outs, states = api.hts_denoise_batch_save(xs, sig, p)
    rng = np.random.default_rng(K)
    gs = [T(rng.normal(size=x.shape)) for x in xs]
    gins = api.hts_denoise_batch_backward(gs, states, p)
    torch.cuda.synchronize()
    for i, (x, s) in enumerate(zip(xs, sig)):
        o, st = api.hts_denoise(x, s, p, save=True)
        assert torch.equal(outs[i], o)
        _state_equal(states[i], st)
        ref, _ = api.hts_denoise_backward(gs[i], st, p)
        assert torch.equal(gins[i], ref)


@pytest.mark.parametrize("C", [1, 3])
def test_batch_with_degenerate_images(C):
    """Images with a single row or column of patch positions, or a 2 x 2
    position grid (every reference has exactly K candidates), batched with
    an ordinary image: each output equals the per-image call bit for bit, and
    the per-image match indices equal the oracle's."""
    p = api.Params(stride=1, window=7, K=4)
    shapes = [(C, 9, 9), (C, 8, 30), (C, 30, 8), (C, 40, 33)]
    ys = [synth.tiny(900 + i, *sh, sigma=15.0, n_blobs=2) for i, sh in enumerate(shapes)]
    sig = [15.0, 10.0, 20.0, 15.0]
    xs = [T(y) for y in ys]
    outs = api.hts_denoise_batch(xs, sig, p)
    torch.cuda.synchronize()
    for i, (y, s) in enumerate(zip(ys, sig)):
        log("degenerate batch", C, shapes[i])
        ref = api.hts_denoise(T(y), s, p)
        assert torch.equal(outs[i], ref)
        assert torch.isfinite(outs[i]).all()
        idx_o, _, _ = omatch.match(y, 8, p.stride, p.window, p.K)
        idx = api.hts_match(T(y), p)
        np.testing.assert_array_equal(idx.cpu().numpy(), idx_o)
