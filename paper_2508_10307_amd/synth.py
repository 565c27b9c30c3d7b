"""Seeded synthetic workloads (inputs only; none of the denoiser's arithmetic).

The paper evaluates on real photographs (Kodak, CC, PolyU, DnD, SIDD, IOCI,
...; dataset table in Sec. IV.B) that are not available here.  These
generators stand in for them with images of the same shapes (256^2, 512^2 and
1024^2 RGB, plus one 24 MPix frame) and value range (0..255), so that block
matching sees realistic structure: smooth blobs, oriented gratings and flat
clipped regions.

Every draw comes from ``numpy.random.default_rng([workload_id, image_index,
stream])`` with stream 0 = clean image, 1 = noise, 2 = per-image size/sigma
draws.  Images are generated in float64 and cast to float32 only after the
noise is added; the noisy image is not clipped.

This module is shared by the oracle tests, the GPU parity tests and the
benchmark, and by nothing else.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SIZES = (256, 384, 512, 768, 1024)


def _rng(workload_id: int, image_index: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(workload_id), int(image_index), int(stream)])


def clean_field(rng: np.random.Generator, H: int, W: int, n_blobs: int) -> np.ndarray:
    """One clean grey field in [0, 255] (float64, H x W).

    Sum of ``n_blobs`` isotropic Gaussian blobs a*exp(-|x-mu|^2/(2 s^2)) with
    a ~ U[0,200], s ~ U[4,30] px, mu uniform over the image (each blob is
    evaluated on its +-6 s support, where it has decayed below 3e-6), plus
    three gratings 20*sin(2 pi <x,(cos t, sin t)>/T + phi) with
    T ~ U[6,40] px, t ~ U[0,pi), phi ~ U[0,2 pi); clipped to [0, 255].
    """
    img = np.zeros((H, W), dtype=np.float64)
    amp = rng.uniform(0.0, 200.0, n_blobs)
    sig = rng.uniform(4.0, 30.0, n_blobs)
    muy = rng.uniform(0.0, H, n_blobs)
    mux = rng.uniform(0.0, W, n_blobs)
    for a, s, my, mx in zip(amp, sig, muy, mux):
        r = 6.0 * s
        y0, y1 = max(0, int(np.floor(my - r))), min(H, int(np.ceil(my + r)) + 1)
        x0, x1 = max(0, int(np.floor(mx - r))), min(W, int(np.ceil(mx + r)) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        gy = np.exp(-((np.arange(y0, y1) - my) ** 2) / (2.0 * s * s))
        gx = np.exp(-((np.arange(x0, x1) - mx) ** 2) / (2.0 * s * s))
        img[y0:y1, x0:x1] += a * np.outer(gy, gx)
    yy = np.arange(H, dtype=np.float64)[:, None]
    xx = np.arange(W, dtype=np.float64)[None, :]
    for _ in range(3):
        T = rng.uniform(6.0, 40.0)
        th = rng.uniform(0.0, np.pi)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        img += 20.0 * np.sin(2.0 * np.pi * (xx * np.cos(th) + yy * np.sin(th)) / T + ph)
    return np.clip(img, 0.0, 255.0)


def clean_image(workload_id: int, image_index: int, C: int, H: int, W: int,
                n_blobs: int) -> np.ndarray:
    """Clean image [C][H][W] float64.  RGB = correlated luminance:
    channel = clip(0.6 L + 0.4 C_ch) with L, C_R, C_G, C_B independent fields."""
    rng = _rng(workload_id, image_index, 0)
    if C == 1:
        return clean_field(rng, H, W, n_blobs)[None]
    L = clean_field(rng, H, W, n_blobs)
    chans = [clean_field(rng, H, W, n_blobs) for _ in range(C)]
    return np.stack([np.clip(0.6 * L + 0.4 * c, 0.0, 255.0) for c in chans])


def clean_video(workload_id: int, T: int, C: int, H: int, W: int, n_blobs: int,
                motion=(1, 2)) -> np.ndarray:
    """T clean frames [T][C][H][W] float64 of one scene under a global
    translation of ``motion`` = (my, mx) pixels per frame: frame t is the
    H x W window at (t my, t mx) of one clean image (clean_image, image
    index 0) of size (H + (T-1) my) x (W + (T-1) mx), so the content of
    frame t reappears in frame t+1 shifted by (-my, -mx)."""
    my, mx = int(motion[0]), int(motion[1])
    base = clean_image(workload_id, 0, C, H + (T - 1) * my, W + (T - 1) * mx, n_blobs)
    return np.stack([base[:, t * my:t * my + H, t * mx:t * mx + W] for t in range(T)])


def add_awgn(workload_id: int, image_index: int, clean: np.ndarray, sigma: float) -> np.ndarray:
    rng = _rng(workload_id, image_index, 1)
    return (clean + rng.normal(0.0, sigma, clean.shape)).astype(np.float32)


def add_poisson_gaussian(workload_id: int, image_index: int, clean: np.ndarray,
                         gain: float = 0.01, read_sigma: float = 10.0):
    """y = gain*Poisson(x/gain) + N(0, read_sigma^2); variance = gain*x + read_sigma^2.
    Returns (noisy float32, sigma) with the per-image scalar noise level
    sigma = sqrt(read_sigma^2 + gain*mean(clean))."""
    rng = _rng(workload_id, image_index, 1)
    y = gain * rng.poisson(clean / gain) + rng.normal(0.0, read_sigma, clean.shape)
    sigma = float(np.sqrt(read_sigma ** 2 + gain * clean.mean()))
    return y.astype(np.float32), sigma


@dataclass
class Params:
    """Method parameters (patch size, reference stride, odd window width,
    group size K, threshold multiplier lambda with tau = lambda*sigma)."""
    ps: int = 8
    stride: int = 3
    window: int = 21
    K: int = 16
    tau_mult: float = 2.7
    gcp_num: int = 6     # gamma = gcp_num/gcp_den = 1.2 (Sec. III.A)
    gcp_den: int = 5


@dataclass
class Image:
    noisy: np.ndarray          # float32 [C][H][W]
    clean: np.ndarray          # float64 [C][H][W]
    sigma: float


@dataclass
class Workload:
    name: str
    params: Params
    images: List[Image] = field(default_factory=list)

    @property
    def mpix(self) -> float:
        return sum(im.noisy.shape[1] * im.noisy.shape[2] for im in self.images) / 1e6


def gray_256(seed: int = 1, H: int = 256, W: int = 256, sigma: float = 25.0) -> Workload:
    """Grey 256x256, 40 blobs, AWGN sigma=25; ps 8, stride 3, window 21, K 16, lambda 2.7."""
    clean = clean_image(seed, 0, 1, H, W, 40)
    return Workload("gray256_awgn25", Params(8, 3, 21, 16, 2.7),
                    [Image(add_awgn(seed, 0, clean, sigma), clean, sigma)])


def rgb_512_pg(seed: int = 2, H: int = 512, W: int = 512) -> Workload:
    """RGB 512x512, 40 blobs per field, Poisson-Gaussian noise (variance 0.01 x + 100);
    ps 8x8x3, stride 3, window 31, K 32."""
    clean = clean_image(seed, 0, 3, H, W, 40)
    noisy, sigma = add_poisson_gaussian(seed, 0, clean)
    return Workload("rgb512_poisson_gauss", Params(8, 3, 31, 32, 2.7),
                    [Image(noisy, clean, sigma)])


def batch64(seed: int = 3, n: int = 64, sizes=SIZES) -> Workload:
    """n RGB images, H and W drawn independently from ``sizes``, AWGN sigma ~ U[5,50];
    parameters as the 512x512 RGB workload."""
    imgs = []
    for i in range(n):
        r = _rng(seed, i, 2)
        H = int(r.choice(sizes))
        W = int(r.choice(sizes))
        sigma = float(r.uniform(5.0, 50.0))
        clean = clean_image(seed, i, 3, H, W, 40)
        imgs.append(Image(add_awgn(seed, i, clean, sigma), clean, sigma))
    return Workload("batch64_rgb_mixed", Params(8, 3, 31, 32, 2.7), imgs)


def large_24mpix(seed: int = 4, H: int = 4000, W: int = 6000) -> Workload:
    """RGB 4000x6000, 400 blobs per field, AWGN sigma=15; stride 2, window 39, K 32."""
    clean = clean_image(seed, 0, 3, H, W, 400)
    return Workload("rgb4000x6000_awgn15", Params(8, 2, 39, 32, 2.7),
                    [Image(add_awgn(seed, 0, clean, 15.0), clean, 15.0)])


def diff_batch16(seed: int = 5, n: int = 16, H: int = 512, W: int = 512) -> Workload:
    """16 RGB 512x512, AWGN sigma=25, K=16 (loss = MSE to the clean image)."""
    imgs = []
    for i in range(n):
        clean = clean_image(seed, i, 3, H, W, 40)
        imgs.append(Image(add_awgn(seed, i, clean, 25.0), clean, 25.0))
    return Workload("batch16_rgb512_grad", Params(8, 3, 31, 16, 2.7), imgs)


def tiny(seed: int, C: int, H: int, W: int, sigma: float = 25.0, n_blobs: int = 4,
         grid: Optional[int] = None) -> np.ndarray:
    """Small noisy image for exhaustive tests.  With ``grid`` the values are
    rounded to multiples of 1/grid (so scaling by 2 stays on the grid)."""
    clean = clean_image(seed, 0, C, H, W, n_blobs)
    y = clean + _rng(seed, 0, 1).normal(0.0, sigma, clean.shape)
    if grid:
        y = np.round(y * grid) / grid
    return y.astype(np.float32)
