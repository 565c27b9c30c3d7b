"""Host-side checks of the C ABI (include/hts.h): the library loads, exports
every declared entry point, and rejects bad arguments with the documented
status before launching anything (no GPU is touched here)."""
import ctypes
import os
import re

import pytest

from oracle.grid import ref_grid as oracle_ref_grid
from paper_2508_10307_amd import _lib as L
from paper_2508_10307_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hts.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hts_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_every_declared_symbol_is_exported_and_bound(lib):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, f"{n} has no ctypes declaration"
    assert set(L.SIGNATURES) == set(names)


def test_version_and_status_strings(lib):
    assert b"gfx950" in lib.hts_version()
    for s in range(5):
        assert lib.hts_status_string(s)
    assert lib.hts_status_string(99) == b"unknown status"


def test_default_params(lib):
    p = L.HtsParams()
    lib.hts_default_params(ctypes.byref(p))
    assert (p.ps, p.stride, p.window, p.K) == (8, 3, 21, 16)
    assert abs(p.tau_mult - 2.7) < 1e-6 and (p.gcp_num, p.gcp_den) == (6, 5)


@pytest.mark.parametrize("H,W,s", [(256, 256, 3), (8, 8, 3), (9, 17, 2), (512, 384, 3),
                                   (4000, 6000, 2), (31, 30, 8)])
def test_ref_grid_matches_oracle(H, W, s):
    p = api.Params(stride=s)
    ny, nx = api.ref_grid(H, W, p)
    _, _, oy, ox = oracle_ref_grid(H, W, 8, s)
    assert (ny, nx) == (oy, ox)


def _ws_status(lib, C=1, H=64, W=64, **kw):
    p = api.Params(**kw).c()
    n = L.c_sz()
    return lib.hts_workspace_size(ctypes.byref(p), C, H, W, ctypes.byref(n)), n.value


@pytest.mark.parametrize("kw,C,HW,status", [
    ({}, 1, (64, 64), L.HTS_OK),
    ({"K": 12}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"K": 1}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"K": 128}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"K": 64}, 3, (64, 64), L.HTS_ERR_UNSUPPORTED),
    ({"K": 64, "window": 21}, 1, (64, 64), L.HTS_OK),
    ({"window": 20}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"window": 65}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"window": 1}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"stride": 0}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"stride": 9}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"ps": 4}, 1, (64, 64), L.HTS_ERR_UNSUPPORTED),
    ({}, 2, (64, 64), L.HTS_OK),                        # spectral tubes
    ({}, 31, (64, 64), L.HTS_OK),
    ({}, 256, (64, 64), L.HTS_OK),
    ({}, 257, (64, 64), L.HTS_ERR_UNSUPPORTED),
    ({"K": 64, "window": 21}, 4, (64, 64), L.HTS_ERR_UNSUPPORTED),
    ({"flags": 1}, 5, (64, 64), L.HTS_ERR_UNSUPPORTED),
    ({}, 0, (64, 64), L.HTS_ERR_UNSUPPORTED),
    ({}, 1, (7, 64), L.HTS_ERR_INVALID),
    ({"K": 32, "window": 7}, 1, (64, 64), L.HTS_ERR_INVALID),   # corner window 4x4 < K
    ({"K": 16, "window": 7}, 1, (64, 64), L.HTS_OK),           # corner window 4x4 = K
    ({"tau_mult": -1.0}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"tau_mult": float("nan")}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"gcp_num": 0}, 3, (64, 64), L.HTS_ERR_INVALID),
    ({"match_mode": 7}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"flags": 4}, 1, (64, 64), L.HTS_ERR_INVALID),
    ({"flags": 3}, 3, (64, 64), L.HTS_OK),
    ({"flags": 1}, 1, (64, 64), L.HTS_OK),
])
def test_parameter_validation(lib, kw, C, HW, status):
    st, n = _ws_status(lib, C, HW[0], HW[1], **kw)
    assert st == status
    if status == L.HTS_OK:
        assert n > 0


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: calls below fail validation first


def test_calls_reject_null_pointers_and_small_workspace(lib):
    p = api.Params().c()
    bp = ctypes.byref(p)
    n = L.c_sz()
    assert lib.hts_workspace_size(bp, 1, 64, 64, ctypes.byref(n)) == L.HTS_OK
    need = n.value
    assert lib.hts_match(bp, None, 1, 64, 64, FAKE, None, None, FAKE, need, None) == L.HTS_ERR_INVALID
    assert lib.hts_match(bp, FAKE, 1, 64, 64, None, None, None, FAKE, need, None) == L.HTS_ERR_INVALID
    assert lib.hts_match(bp, FAKE, 1, 64, 64, FAKE, None, None, FAKE, need - 1, None) == L.HTS_ERR_WORKSPACE
    assert lib.hts_basis(bp, FAKE, 1, 64, 64, None, FAKE, None, None, None, FAKE, need, None) == L.HTS_ERR_INVALID
    assert lib.hts_denoise(bp, FAKE, 1, 64, 64, 25.0, None, None, None, None, None, None, FAKE,
                           need, None) == L.HTS_ERR_INVALID
    assert lib.hts_denoise(bp, FAKE, 1, 64, 64, float("nan"), FAKE, None, None, None, None, None,
                           FAKE, need, None) == L.HTS_ERR_INVALID
    assert lib.hts_denoise(bp, FAKE, 1, 64, 64, -1.0, FAKE, None, None, None, None, None,
                           FAKE, need, None) == L.HTS_ERR_INVALID
    assert lib.hts_denoise(bp, FAKE, 1, 64, 64, 25.0, FAKE, None, None, None, None, None,
                           FAKE, 16, None) == L.HTS_ERR_WORKSPACE
    ny, nx = api.ref_grid(64, 64, api.Params())
    # reference range past the end, num without cnt
    assert lib.hts_filter(bp, FAKE, 1, 64, 64, 25.0, FAKE, FAKE, FAKE, 0, ny * nx + 1, FAKE, FAKE,
                          None, None, FAKE, need, None) == L.HTS_ERR_INVALID
    assert lib.hts_filter(bp, FAKE, 1, 64, 64, 25.0, FAKE, FAKE, FAKE, 0, 4, FAKE, None,
                          None, None, FAKE, need, None) == L.HTS_ERR_INVALID
    assert lib.hts_denoise_backward(bp, FAKE, FAKE, None, FAKE, FAKE, FAKE, 1, 64, 64, FAKE, None,
                                    FAKE, need, None) == L.HTS_ERR_INVALID
    assert lib.hts_aggregate(bp, None, None, 0, 0, 1, 64, 64, None, FAKE, FAKE, None) == L.HTS_ERR_INVALID
    assert lib.hts_denoise_backward_basis(bp, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE, 1, 64,
                                          64, FAKE, FAKE, need, None) == L.HTS_ERR_INVALID
    assert lib.hts_denoise_backward_basis(bp, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 1, 64,
                                          64, FAKE, FAKE, need - 1, None) == L.HTS_ERR_WORKSPACE
    wt = api.Params(flags=L.HTS_FLAG_WEIGHTED).c()
    assert lib.hts_denoise_backward_basis(ctypes.byref(wt), FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE,
                                          FAKE, 1, 64, 64, FAKE, FAKE, need,
                                          None) == L.HTS_ERR_UNSUPPORTED
    # band counts other than 1 and 3: no batch (hts_filter and the adjoint validate as usual)
    assert lib.hts_workspace_size(bp, 5, 64, 64, ctypes.byref(n)) == L.HTS_OK
    need5 = n.value
    assert lib.hts_filter(bp, FAKE, 5, 64, 64, 25.0, None, FAKE, FAKE, 0, 4, FAKE, FAKE,
                          None, None, FAKE, need5, None) == L.HTS_ERR_INVALID
    assert lib.hts_denoise_backward(bp, FAKE, None, FAKE, FAKE, FAKE, FAKE, 5, 64, 64, FAKE, None,
                                    FAKE, need5, None) == L.HTS_ERR_INVALID
    imgs = (L.HtsImage * 1)(L.HtsImage(FAKE.value, FAKE.value, 5, 64, 64, 10.0))
    assert lib.hts_batch_workspace_size(bp, imgs, 1, ctypes.byref(n)) == L.HTS_ERR_UNSUPPORTED
    bad = api.Params(K=12).c()
    assert lib.hts_match(ctypes.byref(bad), FAKE, 1, 64, 64, FAKE, None, None, FAKE, need,
                         None) == L.HTS_ERR_INVALID
    # batched forward with state and batched adjoint: null states or state
    # pointers, and the aggregation / threshold variants without masks
    imgs = (L.HtsImage * 1)(L.HtsImage(FAKE.value, FAKE.value, 3, 64, 64, 10.0))
    good = L.HtsState(FAKE.value, FAKE.value, FAKE.value, FAKE.value, FAKE.value)
    states = (L.HtsState * 1)(good)
    nulls = (L.HtsState * 1)(L.HtsState(FAKE.value, None, FAKE.value, FAKE.value, FAKE.value))
    for fn in (lib.hts_denoise_batch_save, lib.hts_denoise_batch_backward):
        assert fn(bp, imgs, None, 1, FAKE, 1 << 40, None) == L.HTS_ERR_INVALID
        assert fn(bp, imgs, nulls, 1, FAKE, 1 << 40, None) == L.HTS_ERR_INVALID
        assert fn(bp, imgs, states, 0, FAKE, 1 << 40, None) == L.HTS_ERR_INVALID
        for flags in (L.HTS_FLAG_WEIGHTED, L.HTS_FLAG_FOURIER_THRESHOLD):
            pf = api.Params(flags=flags).c()
            assert fn(ctypes.byref(pf), imgs, states, 1, FAKE, 1 << 40,
                      None) == L.HTS_ERR_UNSUPPORTED
        assert fn(bp, imgs, states, 1, FAKE, 16, None) == L.HTS_ERR_WORKSPACE
    # shortlist histogram: null counts or image, small workspace
    sh = lib.hts_batch_shortlist_histogram
    assert sh(bp, imgs, 1, FAKE, 1 << 40, None, None) == L.HTS_ERR_INVALID
    noimg = (L.HtsImage * 1)(L.HtsImage(None, None, 3, 64, 64, 10.0))
    assert sh(bp, noimg, 1, FAKE, 1 << 40, FAKE, None) == L.HTS_ERR_INVALID
    assert sh(bp, imgs, 1, FAKE, 16, FAKE, None) == L.HTS_ERR_WORKSPACE


def test_batch_plan_validation(lib):
    """Batch sizing rejects an empty batch, a null image list, images of
    different channel counts and an image smaller than one patch (no GPU
    call is made)."""
    p = api.Params().c()
    bp = ctypes.byref(p)
    n = L.c_sz()
    one = (L.HtsImage * 1)(L.HtsImage(FAKE.value, FAKE.value, 3, 64, 64, 10.0))
    assert lib.hts_batch_workspace_size(bp, one, 1, ctypes.byref(n)) == L.HTS_OK and n.value > 0
    assert lib.hts_batch_workspace_size(bp, one, 0, ctypes.byref(n)) == L.HTS_ERR_INVALID
    assert lib.hts_batch_workspace_size(bp, None, 1, ctypes.byref(n)) == L.HTS_ERR_INVALID
    mixed = (L.HtsImage * 2)(L.HtsImage(FAKE.value, FAKE.value, 3, 64, 64, 10.0),
                             L.HtsImage(FAKE.value, FAKE.value, 1, 64, 64, 10.0))
    assert lib.hts_batch_workspace_size(bp, mixed, 2, ctypes.byref(n)) == L.HTS_ERR_INVALID
    tiny = (L.HtsImage * 2)(L.HtsImage(FAKE.value, FAKE.value, 3, 64, 64, 10.0),
                            L.HtsImage(FAKE.value, FAKE.value, 3, 7, 64, 10.0))
    assert lib.hts_batch_workspace_size(bp, tiny, 2, ctypes.byref(n)) == L.HTS_ERR_INVALID


def test_workspace_grows_with_image():
    p = api.Params(stride=3, window=31, K=32)
    a = api.workspace_size(p, 3, 256, 256)
    b = api.workspace_size(p, 3, 512, 512)
    assert 3.5 < b / a < 4.5
