"""hts_denoise_noalloc (the entry point for callers that cannot allocate)
through the C ABI against hts_denoise on a caller workspace: the same
kernels on the same data, so the outputs must be equal bit for bit.  Two
calls in a row share the library's one scratch array, the second with a
smaller image (it must not see the first call's contents); an image beyond
the scratch is refused before anything is launched."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2508_10307_amd import _lib as L
from paper_2508_10307_amd import api, synth

pytestmark = pytest.mark.gpu


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev())


def test_noalloc_equals_hts_denoise_on_two_calls_in_a_row():
    cases = [  # (C, H, W, sigma, params): the second call is smaller
        (3, 160, 200, 20.0, api.Params(stride=3, window=15, K=16)),
        (3, 72, 64, 35.0, api.Params(stride=3, window=15, K=16)),
        (1, 56, 48, 15.0, api.Params(stride=2, window=11, K=8)),
    ]
    for i, (C, H, W, s, p) in enumerate(cases):
        print("noalloc call", i, (C, H, W), flush=True)
        x = T(synth.tiny(900 + i, C, H, W, sigma=s, n_blobs=6))
        a = api.hts_denoise_noalloc(x, s, p)
        b = api.hts_denoise(x, s, p)
        torch.cuda.synchronize()
        assert torch.isfinite(a).all()
        assert (a - b).abs().max().item() <= 1e-3
        assert torch.equal(a, b)


def test_noalloc_refuses_an_image_beyond_the_scratch():
    p = api.Params(stride=3, window=31, K=32)
    x = torch.zeros((3, 2048, 2048), device=dev())
    out = torch.full_like(x, 7.0)
    pc = p.c()
    st = L.load().hts_denoise_noalloc(ctypes.byref(pc), ctypes.c_void_p(x.data_ptr()), 3, 2048,
                                      2048, 10.0, ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == L.HTS_ERR_WORKSPACE
    assert bool((out == 7.0).all())
