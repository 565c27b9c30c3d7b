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
