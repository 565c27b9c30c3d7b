"""Pins of the spatio-temporal (video) grouping and denoising in the oracle
(reading V1): one frame, or no temporal reach, reduces to the image
matcher (a separate, vectorised implementation); a static sequence puts the
co-located patches of the neighbouring frames (distance 0) right after the
reference in index order; the truncated temporal window at the ends of the
sequence; sigma = 0 reconstructs; a single frame denoises as an image."""
import numpy as np
import pytest

from oracle import matching, pipeline, video
from paper_2508_10307_amd import synth


def frames_of(T, C, H, W, seed, sigma=20.0):
    return np.stack([synth.tiny(seed + t, C, H, W, sigma=sigma, n_blobs=4) for t in range(T)])


@pytest.mark.parametrize("C", [1, 3, 5])
def test_zero_reach_is_the_image_matcher(C):
    f = frames_of(3, C, 20, 19, 700 + C)
    idx, dist = video.match(f, 8, 3, 9, 8, dt=0)
    n = len(idx) // 3
    H, W = 20, 19
    for t in range(3):
        i1, d1, _ = matching.match(f[t], 8, 3, 9, 8)
        np.testing.assert_array_equal(idx[t * n:(t + 1) * n], i1 + t * H * W)
        np.testing.assert_array_equal(dist[t * n:(t + 1) * n], d1)


def test_one_frame_is_the_image_pipeline():
    f = frames_of(1, 3, 22, 21, 720)
    rv = video.denoise(f, 20.0, 8, 3, 9, 8, dt=2)
    ri = pipeline.denoise(f[0], 20.0, 8, 3, 9, 8)
    np.testing.assert_array_equal(rv["idx"], ri["idx"])
    np.testing.assert_allclose(rv["out"][0], ri["out"], atol=1e-10)


def test_static_sequence_groups_the_co_located_patches_first():
    f = np.repeat(frames_of(1, 1, 20, 20, 730), 4, axis=0)
    idx, dist = video.match(f, 8, 3, 9, 8, dt=1)
    H = W = 20
    n = len(idx) // 4
    for t in range(4):
        for r in range(n):
            row = idx[t * n + r]
            base = int(row[0]) - t * H * W             # the reference's in-frame position
            nb = [t2 for t2 in (t - 1, t + 1) if 0 <= t2 < 4]
            want = sorted((t2 * H * W + base) for t2 in nb)
            assert list(row[1:1 + len(nb)]) == want
            assert (dist[t * n + r, 1:1 + len(nb)] == 0).all()


def test_temporal_window_is_truncated_at_the_ends():
    f = frames_of(3, 1, 18, 18, 740)
    idx, _ = video.match(f, 8, 3, 9, 32, dt=2)
    H = W = 18
    frame_of = idx // (H * W)
    n = len(idx) // 3
    assert set(np.unique(frame_of[:n])) <= {0, 1, 2}
    assert frame_of.max() <= 2 and frame_of.min() >= 0


def test_zero_sigma_reconstructs_the_sequence():
    f = frames_of(3, 3, 20, 21, 750)
    r = video.denoise(f, 0.0, 8, 3, 9, 8, dt=1)
    np.testing.assert_allclose(r["out"], f, atol=1e-9)


def test_synthetic_clip_is_one_translating_scene():
    """The clip generator of the video workloads: frame t+1 is frame t moved
    by the motion vector (content shifted up-left by (my, mx))."""
    from paper_2508_10307_amd import synth
    T, C, H, W, my, mx = 4, 3, 40, 56, 1, 2
    f = synth.clean_video(7, T, C, H, W, 6, motion=(my, mx))
    assert f.shape == (T, C, H, W)
    for t in range(T - 1):
        np.testing.assert_array_equal(f[t + 1][:, :H - my, :W - mx], f[t][:, my:, mx:])
    assert np.abs(f[1] - f[0]).max() > 1.0   # the scene does move
