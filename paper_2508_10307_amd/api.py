"""Python binding of the C ABI (include/hts.h) for torch tensors.

Only argument marshalling happens here: tensors are checked for device,
dtype and contiguity, buffers the C calls write are allocated with torch,
and every step of the method runs in the HIP kernels of libhts.so on the
caller's current stream.  The function names are those of the C ABI.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib as L


@dataclass
class Params:
    """Method parameters (hts_params): patch size, reference stride, odd
    search-window width, group size K (power of two), threshold multiplier
    lambda (tau = lambda * sigma), GCP gamma = gcp_num / gcp_den, distance
    tile mode, flags and launch schedule."""
    ps: int = 8
    stride: int = 3
    window: int = 21
    K: int = 16
    tau_mult: float = 2.7
    gcp_num: int = 6
    gcp_den: int = 5
    match_mode: int = L.HTS_MATCH_BF16
    flags: int = 0
    tune: int = 0

    def c(self) -> L.HtsParams:
        return L.HtsParams(self.ps, self.stride, self.window, self.K, float(self.tau_mult),
                           self.gcp_num, self.gcp_den, self.match_mode, self.flags, self.tune)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _img(x: torch.Tensor, name="noisy") -> torch.Tensor:
    if x.dim() != 3:
        raise ValueError(f"{name} must be [C, H, W]")
    if not x.is_cuda or x.dtype != torch.float32:
        raise ValueError(f"{name} must be a float32 tensor on the GPU")
    return x.contiguous()


def ref_grid(H: int, W: int, p: Params):
    ny, nx = L.c_i32(), L.c_i32()
    pc = p.c()
    L.check("hts_ref_grid", L.load().hts_ref_grid(H, W, ctypes.byref(pc), ctypes.byref(ny),
                                                  ctypes.byref(nx)))
    return ny.value, nx.value


def workspace_size(p: Params, C: int, H: int, W: int) -> int:
    n = L.c_sz()
    pc = p.c()
    L.check("hts_workspace_size", L.load().hts_workspace_size(ctypes.byref(pc), C, H, W,
                                                              ctypes.byref(n)))
    return n.value


def workspace(p: Params, C: int, H: int, W: int, device) -> torch.Tensor:
    return torch.empty(workspace_size(p, C, H, W), dtype=torch.uint8, device=device)


def hts_match(noisy: torch.Tensor, p: Params, want_dist=False, want_green=False, ws=None):
    """Alg. 1 Step 1.  Returns idx int32 [n_ref, K] (and dist int64, green uint8)."""
    x = _img(noisy)
    C, H, W = x.shape
    ny, nx = ref_grid(H, W, p)
    n_ref = ny * nx
    idx = torch.empty((n_ref, p.K), dtype=torch.int32, device=x.device)
    dist = torch.empty((n_ref, p.K), dtype=torch.int64, device=x.device) if want_dist else None
    green = torch.empty(n_ref, dtype=torch.uint8, device=x.device) if want_green else None
    ws = workspace(p, C, H, W, x.device) if ws is None else ws
    pc = p.c()
    L.check("hts_match", L.load().hts_match(ctypes.byref(pc), _ptr(x), C, H, W, _ptr(idx),
                                            _ptr(dist), _ptr(green), _ptr(ws), ws.numel(),
                                            _stream(x.device)))
    out = (idx,)
    if want_dist:
        out += (dist,)
    if want_green:
        out += (green,)
    return out[0] if len(out) == 1 else out


def hts_basis(noisy: torch.Tensor, p: Params, want_fp64=False, ws=None):
    """Alg. 1 Step 2(1).  Returns U, V float32 [C, 8, 8] (+ U64, V64, eig)."""
    x = _img(noisy)
    C, H, W = x.shape
    U = torch.empty((C, 8, 8), dtype=torch.float32, device=x.device)
    V = torch.empty_like(U)
    U64 = V64 = eig = None
    if want_fp64:
        U64 = torch.empty((C, 8, 8), dtype=torch.float64, device=x.device)
        V64 = torch.empty_like(U64)
        eig = torch.empty((2, C // 2 + 1, 8), dtype=torch.float64, device=x.device)
    ws = workspace(p, C, H, W, x.device) if ws is None else ws
    pc = p.c()
    L.check("hts_basis", L.load().hts_basis(ctypes.byref(pc), _ptr(x), C, H, W, _ptr(U), _ptr(V),
                                            _ptr(U64), _ptr(V64), _ptr(eig), _ptr(ws), ws.numel(),
                                            _stream(x.device)))
    return (U, V, U64, V64, eig) if want_fp64 else (U, V)


def mask_words(n_groups: int, K: int, C: int) -> int:
    return (n_groups * K * C * 64 + 31) // 32


def hts_filter(noisy, sigma, idx, U, V, p: Params, ref_begin=0, ref_count=None,
               accumulate=True, want_group_est=False, want_masks=False, ws=None):
    """Alg. 1 Step 2(2)-(4) for references [ref_begin, ref_begin + ref_count).
    Returns a dict with num, cnt (when accumulate), group_est, masks."""
    x = _img(noisy)
    C, H, W = x.shape
    n_ref = idx.shape[0]
    ref_count = n_ref - ref_begin if ref_count is None else ref_count
    dev = x.device
    num = torch.zeros((C, H, W), dtype=torch.float32, device=dev) if accumulate else None
    cnt = torch.zeros((H, W), dtype=torch.float32, device=dev) if accumulate else None
    est = (torch.empty((ref_count, p.K, C, 8, 8), dtype=torch.float32, device=dev)
           if want_group_est else None)
    masks = (torch.zeros(mask_words(ref_count, p.K, C), dtype=torch.int32, device=dev)
             if want_masks else None)
    ws = workspace(p, C, H, W, dev) if ws is None else ws
    pc = p.c()
    idx = idx.contiguous()
    L.check("hts_filter", L.load().hts_filter(
        ctypes.byref(pc), _ptr(x), C, H, W, float(sigma), _ptr(idx), _ptr(U.contiguous()),
        _ptr(V.contiguous()), ref_begin, ref_count, _ptr(num), _ptr(cnt), _ptr(est), _ptr(masks),
        _ptr(ws), ws.numel(), _stream(dev)))
    return {"num": num, "cnt": cnt, "group_est": est, "masks": masks}


def hts_aggregate(p: Params, C, H, W, num, cnt, group_est=None, idx=None, ref_begin=0,
                  ref_count=0, out=None):
    """Eq. 2: add group estimates into num/cnt and/or finalise out = num / cnt."""
    pc = p.c()
    dev = num.device
    L.check("hts_aggregate", L.load().hts_aggregate(
        ctypes.byref(pc), _ptr(group_est), _ptr(idx), ref_begin, ref_count, C, H, W, _ptr(num),
        _ptr(cnt), _ptr(out), _stream(dev)))
    return out


def new_state(p: Params, C: int, H: int, W: int, dev) -> dict:
    """Device buffers for one image's backward state: dict(idx, masks, U, V,
    cnt) in the layouts of hts_state."""
    ny, nx = ref_grid(H, W, p)
    n_ref = ny * nx
    return {"idx": torch.empty((n_ref, p.K), dtype=torch.int32, device=dev),
            "masks": torch.zeros(mask_words(n_ref, p.K, C), dtype=torch.int32, device=dev),
            "U": torch.empty((C, 8, 8), dtype=torch.float32, device=dev),
            "V": torch.empty((C, 8, 8), dtype=torch.float32, device=dev),
            "cnt": torch.empty((H, W), dtype=torch.float32, device=dev)}


def _states(states) -> "ctypes.Array":
    arr = (L.HtsState * len(states))()
    for i, st in enumerate(states):
        arr[i] = L.HtsState(st["idx"].data_ptr(), st["masks"].data_ptr(), st["U"].data_ptr(),
                            st["V"].data_ptr(), st["cnt"].data_ptr())
    return arr


def hts_denoise(noisy, sigma, p: Params, save=False, ws=None):
    """Algorithm 1 end to end.  With save=True also returns the state the
    adjoint needs: dict(idx, masks, U, V, cnt)."""
    x = _img(noisy)
    C, H, W = x.shape
    dev = x.device
    out = torch.empty_like(x)
    st = new_state(p, C, H, W, dev) if save else None
    g = st or {}
    ws = workspace(p, C, H, W, dev) if ws is None else ws
    pc = p.c()
    L.check("hts_denoise", L.load().hts_denoise(
        ctypes.byref(pc), _ptr(x), C, H, W, float(sigma), _ptr(out), _ptr(g.get("idx")),
        _ptr(g.get("masks")), _ptr(g.get("U")), _ptr(g.get("V")), _ptr(g.get("cnt")), _ptr(ws),
        ws.numel(), _stream(dev)))
    return (out, st) if save else out


def hts_denoise_backward(grad_out, st, p: Params, ws=None):
    """Adjoint with frozen idx / masks / basis / counts.  Returns
    (grad_noisy, grad_tau_mult) - the latter is identically zero."""
    g = _img(grad_out, "grad_out")
    C, H, W = g.shape
    dev = g.device
    gin = torch.empty_like(g)
    gtau = torch.empty(1, dtype=torch.float32, device=dev)
    ws = workspace(p, C, H, W, dev) if ws is None else ws
    pc = p.c()
    L.check("hts_denoise_backward", L.load().hts_denoise_backward(
        ctypes.byref(pc), _ptr(g), _ptr(st["idx"]), _ptr(st["masks"]), _ptr(st["U"]),
        _ptr(st["V"]), _ptr(st["cnt"]), C, H, W, _ptr(gin), _ptr(gtau), _ptr(ws), ws.numel(),
        _stream(dev)))
    return gin, gtau


def hts_denoise_noalloc(noisy: torch.Tensor, sigma: float, p: Params, out=None):
    """hts_denoise on the library's fixed device scratch (no workspace)."""
    x = _img(noisy)
    C, H, W = x.shape
    out = torch.empty_like(x) if out is None else out
    pc = p.c()
    L.check("hts_denoise_noalloc", L.load().hts_denoise_noalloc(
        ctypes.byref(pc), _ptr(x), C, H, W, float(sigma), _ptr(out), _stream(x.device)))
    return out


def hts_match_fallback_count(p: Params, C: int, H: int, W: int, ws: torch.Tensor) -> torch.Tensor:
    """References of the last hts_match / hts_denoise on workspace ws whose
    certified shortlist overflowed (matched by the exact window scan).
    Returns a device int32 tensor [1]."""
    out = torch.empty(1, dtype=torch.int32, device=ws.device)
    pc = p.c()
    L.check("hts_match_fallback_count", L.load().hts_match_fallback_count(
        ctypes.byref(pc), C, H, W, _ptr(ws), ws.numel(), _ptr(out), _stream(ws.device)))
    return out


def hts_batch_fallback_counts(p: Params, noisy, outs, sigmas, ws: torch.Tensor) -> torch.Tensor:
    """The same per image of the last hts_denoise_batch on ws with these
    images.  Returns a device int32 tensor [n]."""
    arr = _images(noisy, outs, sigmas)
    out = torch.empty(len(noisy), dtype=torch.int32, device=ws.device)
    pc = p.c()
    L.check("hts_batch_fallback_counts", L.load().hts_batch_fallback_counts(
        ctypes.byref(pc), arr, len(noisy), _ptr(ws), ws.numel(), _ptr(out), _stream(ws.device)))
    return out


def hts_batch_shortlist_histogram(p: Params, noisy, ws: Optional[torch.Tensor] = None):
    """Shortlist sizes of the certified match over a batch: a device int32
    tensor [HTS_SHORTLIST_BINS]; entry s <= 128 counts the references whose
    shortlist held s candidates, the last entry the overflows."""
    xs = [_img(x) for x in noisy]
    dev = xs[0].device
    sig = [0.0] * len(xs)
    if ws is None:
        ws = torch.empty(batch_workspace_size(p, xs, xs, sig), dtype=torch.uint8, device=dev)
    arr = _images(xs, xs, sig)
    out = torch.empty(L.HTS_SHORTLIST_BINS, dtype=torch.int32, device=dev)
    pc = p.c()
    L.check("hts_batch_shortlist_histogram", L.load().hts_batch_shortlist_histogram(
        ctypes.byref(pc), arr, len(xs), _ptr(ws), ws.numel(), _ptr(out), _stream(dev)))
    return out


def _images(noisy: Sequence[torch.Tensor], outs: Sequence[torch.Tensor], sigmas):
    arr = (L.HtsImage * len(noisy))()
    for i, (x, o, s) in enumerate(zip(noisy, outs, sigmas)):
        C, H, W = x.shape
        arr[i] = L.HtsImage(x.data_ptr(), o.data_ptr(), C, H, W, float(s))
    return arr


def batch_workspace_size(p: Params, noisy, outs, sigmas) -> int:
    arr = _images(noisy, outs, sigmas)
    n = L.c_sz()
    pc = p.c()
    L.check("hts_batch_workspace_size", L.load().hts_batch_workspace_size(
        ctypes.byref(pc), arr, len(noisy), ctypes.byref(n)))
    return n.value


def hts_denoise_batch(noisy: List[torch.Tensor], sigmas, p: Params, outs=None, ws=None):
    """Algorithm 1 for a list of images of any sizes / noise levels (one
    persistent, graph-captured pipeline).  Returns the list of outputs."""
    xs = [_img(x) for x in noisy]
    dev = xs[0].device
    outs = [torch.empty_like(x) for x in xs] if outs is None else outs
    if ws is None:
        ws = torch.empty(batch_workspace_size(p, xs, outs, sigmas), dtype=torch.uint8, device=dev)
    arr = _images(xs, outs, sigmas)
    pc = p.c()
    L.check("hts_denoise_batch", L.load().hts_denoise_batch(
        ctypes.byref(pc), arr, len(xs), _ptr(ws), ws.numel(), _stream(dev)))
    return outs


def hts_denoise_batch_save(noisy: List[torch.Tensor], sigmas, p: Params, outs=None, states=None,
                           ws=None):
    """hts_denoise_batch that also writes each image's backward state.
    Returns (outs, states), states a list of dicts as new_state makes."""
    xs = [_img(x) for x in noisy]
    dev = xs[0].device
    outs = [torch.empty_like(x) for x in xs] if outs is None else outs
    if states is None:
        states = [new_state(p, *x.shape, dev) for x in xs]
    if ws is None:
        ws = torch.empty(batch_workspace_size(p, xs, outs, sigmas), dtype=torch.uint8, device=dev)
    arr = _images(xs, outs, sigmas)
    sarr = _states(states)
    pc = p.c()
    L.check("hts_denoise_batch_save", L.load().hts_denoise_batch_save(
        ctypes.byref(pc), arr, sarr, len(xs), _ptr(ws), ws.numel(), _stream(dev)))
    return outs, states


def hts_denoise_batch_backward(grads: List[torch.Tensor], states, p: Params, grad_ins=None,
                               ws=None):
    """Frozen-map adjoint of a batch (hts_denoise_backward per image, in one
    graph-captured pipeline).  Returns the list of input gradients."""
    gs = [_img(g, "grad_out") for g in grads]
    dev = gs[0].device
    grad_ins = [torch.empty_like(g) for g in gs] if grad_ins is None else grad_ins
    sig = [0.0] * len(gs)
    if ws is None:
        ws = torch.empty(batch_workspace_size(p, gs, grad_ins, sig), dtype=torch.uint8, device=dev)
    arr = _images(gs, grad_ins, sig)
    sarr = _states(states)
    pc = p.c()
    L.check("hts_denoise_batch_backward", L.load().hts_denoise_batch_backward(
        ctypes.byref(pc), arr, sarr, len(gs), _ptr(ws), ws.numel(), _stream(dev)))
    return grad_ins


BATCH_STAGES = ("prep", "match", "cov", "basis", "filter", "finalize")


def hts_denoise_batch_staged(noisy: List[torch.Tensor], sigmas, p: Params, outs, ws,
                             events: Sequence["torch.cuda.Event"]):
    """hts_denoise_batch launched stage by stage on the current stream,
    recording the 7 timing events (torch.cuda.Event(enable_timing=True)) at
    the stage boundaries; stage i lasts events[i] -> events[i + 1]
    (BATCH_STAGES)."""
    xs = [_img(x) for x in noisy]
    dev = xs[0].device
    for e in events:   # torch creates the HIP event lazily, on first record
        e.record()
    arr = _images(xs, outs, sigmas)
    evs = (L.c_vp * len(events))(*[ctypes.c_void_p(e.cuda_event) for e in events])
    pc = p.c()
    L.check("hts_denoise_batch_staged", L.load().hts_denoise_batch_staged(
        ctypes.byref(pc), arr, len(xs), _ptr(ws), ws.numel(), _stream(dev), evs, len(events)))
    return outs


def _samples(samples, n_rows: int, dev) -> torch.Tensor:
    t = torch.as_tensor(samples, dtype=torch.int32)
    if t.dim() == 1:
        t = t.reshape(1, -1)
    if t.shape[0] != n_rows or t.shape[1] < 1:
        raise ValueError("samples must be [n_images, n_samples] reference indices")
    return t.to(dev).contiguous()


def hts_adapt_sigma(noisy: torch.Tensor, idx: torch.Tensor, samples, sigma_est: float,
                    p: Params, beta: float = 1.2, gamma: int = 13):
    """A-Haar-tSVD noise-level adjustment of one image (Eq. 21-22) for a
    caller-supplied sigma_est: the sampled groups' eigenvalue ranks and the
    voted sigma-hat.  Returns (sigma_hat [1] tensor, ranks [n_samples])."""
    x = _img(noisy)
    dev = x.device
    C, H, W = x.shape
    if not idx.is_cuda or idx.dtype != torch.int32:
        raise ValueError("idx must be an int32 tensor on the GPU")
    smp = _samples(samples, 1, dev)
    n = smp.shape[1]
    sig = torch.empty(1, dtype=torch.float32, device=dev)
    ranks = torch.empty(n, dtype=torch.int32, device=dev)
    pc = p.c()
    L.check("hts_adapt_sigma", L.load().hts_adapt_sigma(
        ctypes.byref(pc), _ptr(x), C, H, W, _ptr(idx.contiguous()), _ptr(smp), n,
        float(sigma_est), float(beta), int(gamma), _ptr(ranks), _ptr(sig), _stream(dev)))
    return sig, ranks


def hts_denoise_batch_adaptive(noisy: List[torch.Tensor], sigma_est, samples, p: Params,
                               beta: float = 1.2, gamma: int = 13, outs=None, ws=None):
    """A-Haar-tSVD over a batch (each image, e.g. each sub-image of a
    picture, adjusts its own sigma_est from its sampled groups, samples =
    [n_images, n_samples] reference indices, then is denoised with it).
    Returns (outputs, sigma_hat [n], ranks [n, n_samples])."""
    xs = [_img(x) for x in noisy]
    dev = xs[0].device
    outs = [torch.empty_like(x) for x in xs] if outs is None else outs
    if ws is None:
        ws = torch.empty(batch_workspace_size(p, xs, outs, sigma_est), dtype=torch.uint8,
                         device=dev)
    smp = _samples(samples, len(xs), dev)
    ns = smp.shape[1]
    sig = torch.empty(len(xs), dtype=torch.float32, device=dev)
    ranks = torch.empty(len(xs), ns, dtype=torch.int32, device=dev)
    arr = _images(xs, outs, sigma_est)
    pc = p.c()
    L.check("hts_denoise_batch_adaptive", L.load().hts_denoise_batch_adaptive(
        ctypes.byref(pc), arr, len(xs), _ptr(smp), ns, float(beta), int(gamma), _ptr(ranks),
        _ptr(sig), _ptr(ws), ws.numel(), _stream(dev)))
    return outs, sig, ranks


def sub_images(H: int, W: int, sub_h: int, sub_w: int):
    """Tiling of an H x W image into sub-images of about sub_h x sub_w
    (Algorithm A-Haar-tSVD): max(1, H // sub_h) rows and max(1, W // sub_w)
    columns of near-equal tiles, each at least sub_h x sub_w unless the image
    is smaller.  Returns [(y0, x0, h, w)]."""
    ny, nx = max(1, H // sub_h), max(1, W // sub_w)
    ys = [round(i * H / ny) for i in range(ny + 1)]
    xs = [round(j * W / nx) for j in range(nx + 1)]
    return [(ys[i], xs[j], ys[i + 1] - ys[i], xs[j + 1] - xs[j])
            for i in range(ny) for j in range(nx)]


def draw_samples(subs, p: Params, n_samples: int, seed: int = 0):
    """The random choice of the sampled groups (references drawn without
    replacement, numpy generator seeded with [seed, sub-image]); an input of
    the adjustment, so that a caller can reproduce it."""
    import numpy as np
    rows = []
    for i, (_, _, h, w) in enumerate(subs):
        ny, nx = ref_grid(h, w, p)
        rng = np.random.default_rng([seed, i])
        n = ny * nx
        rows.append(rng.choice(n, size=n_samples, replace=n < n_samples).astype(np.int32))
    return np.stack(rows)


def a_haar_tsvd(x: torch.Tensor, sigma_est: float, sub=(256, 256), n_samples: int = 16,
                seed: int = 0, beta: float = 1.2, gamma: int = 13, **params):
    """A-Haar-tSVD of one [C, H, W] image with a caller-supplied sigma_est:
    the image is split into sub-images, each adjusts sigma_est from its own
    sampled groups and is denoised with it, all in one adaptive batch.
    Returns (denoised image, sigma_hat per sub-image, sub-image list)."""
    x = _img(x)
    p = Params(**params)
    C, H, W = x.shape
    subs = sub_images(H, W, sub[0], sub[1])
    parts = [x[:, y0:y0 + h, x0:x0 + w].contiguous() for (y0, x0, h, w) in subs]
    smp = draw_samples(subs, p, n_samples, seed)
    outs, sig, _ = hts_denoise_batch_adaptive(parts, [sigma_est] * len(parts), smp, p, beta,
                                              gamma)
    out = torch.empty_like(x)
    for (y0, x0, h, w), o in zip(subs, outs):
        out[:, y0:y0 + h, x0:x0 + w] = o
    return out, sig, subs


def hts_autotune(p: Params, C, H, W, cache_path: Optional[str] = None, device="cuda"):
    """Time the launch schedules for this shape on the GPU; returns the tune word."""
    size = workspace_size(p, C, H, W) + 2 * C * H * W * 4 + (H * W) * p.K * 4 + (1 << 20)
    ws = torch.empty(size, dtype=torch.uint8, device=device)
    out = L.c_i32()
    pc = p.c()
    L.check("hts_autotune", L.load().hts_autotune(
        ctypes.byref(pc), C, H, W, cache_path.encode() if cache_path else None,
        ctypes.byref(out), _ptr(ws), ws.numel(), _stream(torch.device(device))))
    return out.value


def hts_denoise_grad_tau(noisy, grad_out, st, sigma: float, p: Params, kappa: float = 0.1,
                         ws=None):
    """Surrogate derivative of a loss with respect to tau_mult (logistic
    relaxation of the keep-mask, width kappa * sigma), with the grouping,
    basis and coverage count st of hts_denoise(save=True) frozen.  Returns a
    device scalar tensor [1]."""
    x = _img(noisy)
    g = _img(grad_out, "grad_out")
    C, H, W = x.shape
    dev = x.device
    out = torch.empty(1, dtype=torch.float32, device=dev)
    ws = workspace(p, C, H, W, dev) if ws is None else ws
    pc = p.c()
    L.check("hts_denoise_grad_tau", L.load().hts_denoise_grad_tau(
        ctypes.byref(pc), _ptr(x), _ptr(g), _ptr(st["idx"]), _ptr(st["U"]), _ptr(st["V"]),
        _ptr(st["cnt"]), C, H, W, float(sigma), float(kappa), _ptr(out), _ptr(ws), ws.numel(),
        _stream(dev)))
    return out


def hts_denoise_backward_basis(noisy, grad_out, st, p: Params, grad_in, basis64=None, ws=None):
    """Adds into grad_in the derivative through the learned basis (with the
    grouping, masks and counts of st frozen): the part of dL/dnoisy that
    flows through U(noisy), V(noisy).  basis64 = (U64, V64, eig) of
    hts_basis(noisy, p, want_fp64=True), computed here when None.  Returns
    grad_in."""
    x = _img(noisy)
    g = _img(grad_out, "grad_out")
    C, H, W = x.shape
    dev = x.device
    if basis64 is None:
        basis64 = hts_basis(x, p, want_fp64=True)[2:]
    U64, V64, eig = basis64
    ws = workspace(p, C, H, W, dev) if ws is None else ws
    pc = p.c()
    L.check("hts_denoise_backward_basis", L.load().hts_denoise_backward_basis(
        ctypes.byref(pc), _ptr(x), _ptr(g), _ptr(st["idx"]), _ptr(st["masks"]), _ptr(U64),
        _ptr(V64), _ptr(eig), _ptr(st["cnt"]), C, H, W, _ptr(grad_in), _ptr(ws), ws.numel(),
        _stream(dev)))
    return grad_in


def video_workspace_size(p: Params, T: int, C: int, H: int, W: int, dt: int) -> int:
    """hts_video_workspace_size: bytes of the workspace of a T-frame clip."""
    pc = p.c()
    n = L.c_sz()
    L.check("hts_video_workspace_size", L.load().hts_video_workspace_size(
        ctypes.byref(pc), T, C, H, W, int(dt), ctypes.byref(n)))
    return n.value


def hts_denoise_video(frames: torch.Tensor, sigma: float, p: Params, dt: int = 1, save=False,
                      ws=None):
    """Video denoising with spatio-temporal search over frames t-dt..t+dt.
    frames [T, C, H, W] float32 on the GPU.  With save=True also returns
    dict(idx [T n_ref, K] in stacked coordinates, masks, U, V, cnt [T H, W])."""
    if frames.dim() != 4:
        raise ValueError("frames must be [T, C, H, W]")
    if not frames.is_cuda or frames.dtype != torch.float32:
        raise ValueError("frames must be a float32 tensor on the GPU")
    x = frames.contiguous()
    T, C, H, W = x.shape
    dev = x.device
    out = torch.empty_like(x)
    pc = p.c()
    n = L.c_sz()
    L.check("hts_video_workspace_size", L.load().hts_video_workspace_size(
        ctypes.byref(pc), T, C, H, W, int(dt), ctypes.byref(n)))
    if ws is None:
        ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
    st = {}
    if save:
        ny, nx = ref_grid(H, W, p)
        n_ref = T * ny * nx
        st = {"idx": torch.empty((n_ref, p.K), dtype=torch.int32, device=dev),
              "masks": torch.zeros(mask_words(n_ref, p.K, C), dtype=torch.int32, device=dev),
              "U": torch.empty((C, 8, 8), dtype=torch.float32, device=dev),
              "V": torch.empty((C, 8, 8), dtype=torch.float32, device=dev),
              "cnt": torch.empty((T * H, W), dtype=torch.float32, device=dev)}
    L.check("hts_denoise_video", L.load().hts_denoise_video(
        ctypes.byref(pc), _ptr(x), T, C, H, W, int(dt), float(sigma), _ptr(out),
        _ptr(st.get("idx")), _ptr(st.get("masks")), _ptr(st.get("U")), _ptr(st.get("V")),
        _ptr(st.get("cnt")), _ptr(ws), ws.numel(), _stream(dev)))
    return (out, st) if save else out


def hts_denoise_video_backward(grad_out: torch.Tensor, st, p: Params, dt: int = 1, ws=None):
    """Adjoint of hts_denoise_video with the state st of the forward call
    (save=True) frozen.  Returns grad_noisy [T, C, H, W]."""
    g = grad_out.contiguous()
    if g.dim() != 4 or not g.is_cuda or g.dtype != torch.float32:
        raise ValueError("grad_out must be a float32 [T, C, H, W] tensor on the GPU")
    T, C, H, W = g.shape
    dev = g.device
    pc = p.c()
    if ws is None:
        n = L.c_sz()
        L.check("hts_video_workspace_size", L.load().hts_video_workspace_size(
            ctypes.byref(pc), T, C, H, W, int(dt), ctypes.byref(n)))
        ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
    gin = torch.empty_like(g)
    L.check("hts_denoise_video_backward", L.load().hts_denoise_video_backward(
        ctypes.byref(pc), _ptr(g), T, C, H, W, int(dt), _ptr(st["idx"]), _ptr(st["masks"]),
        _ptr(st["U"]), _ptr(st["V"]), _ptr(st["cnt"]), _ptr(gin), _ptr(ws), ws.numel(),
        _stream(dev)))
    return gin


class HaarTSVD(torch.autograd.Function):
    """Differentiable Haar-tSVD denoiser: forward = hts_denoise; backward =
    the hand-written adjoint kernel with match indices, threshold masks,
    basis and coverage counts frozen at the forward pass; with
    basis_grad=True it adds the derivative through the learned basis
    (hts_denoise_backward_basis).  The exact gradient with respect to the
    threshold multiplier is zero (it only moves the frozen masks); with
    tau_kappa > 0 the backward returns instead the surrogate derivative of
    hts_denoise_grad_tau (relaxation width tau_kappa * sigma)."""

    @staticmethod
    def forward(ctx, noisy, sigma, tau_mult, p: Params, tau_kappa: float = 0.0,
                basis_grad: bool = False):
        q = Params(**{**p.__dict__, "tau_mult": float(tau_mult)})
        x = noisy.detach()
        out, st = hts_denoise(x, float(sigma), q, save=True)
        ctx.st = st
        ctx.p = q
        ctx.sigma = float(sigma)
        ctx.kappa = float(tau_kappa)
        ctx.basis_grad = bool(basis_grad)
        ctx.noisy = x if (ctx.kappa > 0 or ctx.basis_grad) else None
        return out

    @staticmethod
    def backward(ctx, grad):
        g = grad.contiguous()
        gin, gtau = hts_denoise_backward(g, ctx.st, ctx.p)
        if ctx.basis_grad:
            hts_denoise_backward_basis(ctx.noisy, g, ctx.st, ctx.p, gin)
        if ctx.kappa > 0:
            gtau = hts_denoise_grad_tau(ctx.noisy, g, ctx.st, ctx.sigma, ctx.p, ctx.kappa)
        return gin, None, gtau.reshape(()) if ctx.needs_input_grad[2] else None, None, None, None


class HaarTSVDBatch(torch.autograd.Function):
    """HaarTSVD over a batch [N, C, H, W] with one noise level per image:
    forward = hts_denoise_batch_save, backward = hts_denoise_batch_backward
    (one graph-captured pipeline each way), the same values as HaarTSVD per
    image.  tau_mult is shared by the batch: with tau_kappa > 0 its
    surrogate derivative is the sum of the images' hts_denoise_grad_tau;
    basis_grad=True adds each image's derivative through its basis."""

    @staticmethod
    def forward(ctx, noisy, sigmas, tau_mult, p: Params, tau_kappa: float = 0.0,
                basis_grad: bool = False):
        q = Params(**{**p.__dict__, "tau_mult": float(tau_mult)})
        x = noisy.detach()
        if x.dim() != 4:
            raise ValueError("noisy must be [N, C, H, W]")
        x = x.contiguous()
        sig = [float(v) for v in torch.as_tensor(sigmas, dtype=torch.float64).reshape(-1).tolist()]
        if len(sig) == 1:
            sig = sig * x.shape[0]
        if len(sig) != x.shape[0]:
            raise ValueError("one sigma per image")
        out = torch.empty_like(x)
        _, st = hts_denoise_batch_save(list(x.unbind(0)), sig, q, outs=list(out.unbind(0)))
        ctx.st, ctx.p, ctx.sig = st, q, sig
        ctx.kappa = float(tau_kappa)
        ctx.basis_grad = bool(basis_grad)
        ctx.noisy = x if (ctx.kappa > 0 or ctx.basis_grad) else None
        return out

    @staticmethod
    def backward(ctx, grad):
        g = grad.contiguous()
        gin = torch.empty_like(g)
        gs, gi = list(g.unbind(0)), list(gin.unbind(0))
        hts_denoise_batch_backward(gs, ctx.st, ctx.p, grad_ins=gi)
        gtau = torch.zeros(1, dtype=torch.float32, device=g.device)
        for i in range(len(gs)):
            if ctx.basis_grad:
                hts_denoise_backward_basis(ctx.noisy[i], gs[i], ctx.st[i], ctx.p, gi[i])
            if ctx.kappa > 0:
                gtau += hts_denoise_grad_tau(ctx.noisy[i], gs[i], ctx.st[i], ctx.sig[i], ctx.p,
                                             ctx.kappa)
        return gin, None, gtau.reshape(()) if ctx.needs_input_grad[2] else None, None, None, None


def denoise(x: torch.Tensor, sigma: float, **params) -> torch.Tensor:
    """Convenience: denoise one [C, H, W] float32 GPU image."""
    return hts_denoise(x, sigma, Params(**params))
