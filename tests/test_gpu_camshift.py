"""GPU parity of the colour likelihood (Eq. 2.18-2.21), the moment integral
images and CAMSHIFT (Alg. 1) against the CPU oracle: likelihood codes and
moment images bit-exact (the latter modulo 2^32 where stored so), likelihoods
equal to the oracle's FP64 ratio rounded to FP32, CAMSHIFT centres and step
counts identical (the oracle sums each window directly)."""
import numpy as np
import pytest
import torch

import oracle
from synth.video import config5

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def ihlib():
    import paper_1711_01656_amd as ih
    return ih


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(*a):
    print(*a, flush=True)


def mod32(a):
    return np.asarray(a).astype(np.int64) & 0xFFFFFFFF


def few_colours(seed, H, W, levels=6):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, levels, size=(3, H, W)) * (255 // (levels - 1))).astype(np.uint8)


@pytest.mark.parametrize("H,W,fg,bg", [
    (60, 80, (20, 30, 40, 55), (10, 15, 52, 72)),
    (1, 1, (0, 0, 1, 1), (0, 0, 1, 1)),
    (97, 131, (0, 0, 97, 131), (0, 0, 97, 131)),          # no background pixels
    (50, 50, (10, 10, 10, 30), (0, 0, 50, 50)),           # empty foreground
    (70, 90, (30, 40, 60, 85), (0, 0, 45, 60)),           # fg not inside bg
])
def test_color_likelihood_matches_oracle(H, W, fg, bg):
    ih = ihlib()
    rgb = few_colours(H * W, H, W)
    q, L = ih.ih_color_likelihood(gpu(rgb), fg, bg)
    oq, oL = oracle.color_likelihood(rgb, fg, bg)
    assert np.array_equal(q.cpu().numpy(), oq)
    assert np.array_equal(L.cpu().numpy(), oL.astype(np.float32))


def test_color_likelihood_many_colours_and_reuse():
    ih = ihlib()
    rng = np.random.default_rng(3)
    H, W = 300, 400
    rgb = rng.integers(0, 256, size=(3, H, W)).astype(np.uint8)
    ws = torch.empty(ih.lib().ih_color_likelihood_workspace_size(), dtype=torch.uint8, device=DEV)
    t = gpu(rgb)
    for fg, bg in (((100, 150, 200, 250), (50, 100, 250, 300)), ((0, 0, 150, 200), (0, 0, 300, 400))):
        q, L = ih.ih_color_likelihood(t, fg, bg, ws=ws)         # the workspace is cleared every call
        oq, oL = oracle.color_likelihood(rgb, fg, bg)
        assert np.array_equal(q.cpu().numpy(), oq)
        assert np.array_equal(L.cpu().numpy(), oL.astype(np.float32))


@pytest.mark.parametrize("H,W", [(1, 1), (1, 300), (300, 1), (97, 203), (720, 1280)])
def test_moment_images_match_oracle(H, W):
    ih = ihlib()
    q = np.random.default_rng(H + W).integers(0, 256, size=(H, W)).astype(np.uint8)
    S, Sx, Sy = ih.ih_moment_images(gpu(q))
    oS, oSx, oSy = oracle.moment_images(q)
    assert np.array_equal(S.cpu().numpy(), oS)
    assert np.array_equal(mod32(Sx.cpu().numpy()), mod32(oSx))
    assert np.array_equal(mod32(Sy.cpu().numpy()), mod32(oSy))


def test_moment_images_tile_shapes():
    ih = ihlib()
    H, W = 150, 333
    q = np.random.default_rng(4).integers(0, 256, size=(H, W)).astype(np.uint8)
    oS, oSx, oSy = oracle.moment_images(q)
    t = gpu(q)
    for th in (1, 7, 32, 128):
        for tw in (64, 128, 256):
            if th * tw > 32768 or th * (tw + 4) * 2 > 64 * 1024 - 8 * max(th, tw):
                continue
            S, Sx, Sy = ih.ih_moment_images(t, cfg=ih.TileCfg(th, tw, 1))
            assert np.array_equal(S.cpu().numpy(), oS), (th, tw)
            assert np.array_equal(mod32(Sx.cpu().numpy()), mod32(oSx)), (th, tw)
            assert np.array_equal(mod32(Sy.cpu().numpy()), mod32(oSy)), (th, tw)


def blob_map(H, W, seed):
    rng = np.random.default_rng(seed)
    r = np.arange(H)[:, None]
    c = np.arange(W)[None, :]
    q = rng.integers(0, 40, size=(H, W)).astype(np.float64)
    for _ in range(6):
        cr, cc, s = rng.uniform(0, H), rng.uniform(0, W), rng.uniform(5, 25)
        q += 200 * np.exp(-((r - cr) ** 2 + (c - cc) ** 2) / (2 * s * s))
    return np.clip(q, 0, 255).astype(np.uint8)


@pytest.mark.parametrize("H,W,wh,ww,delta,max_iter", [
    (120, 160, 31, 31, 0.5, 20), (200, 150, 40, 64, 0.1, 50), (64, 64, 64, 64, 0.5, 10),
    (90, 110, 1, 1, 0.5, 5), (300, 400, 101, 81, 0.25, 30)])
def test_camshift_matches_oracle(H, W, wh, ww, delta, max_iter):
    ih = ihlib()
    q = blob_map(H, W, H + wh)
    rng = np.random.default_rng(W + ww)
    starts = np.stack([rng.uniform(-5, H + 5, 3000), rng.uniform(-5, W + 5, 3000)], 1)
    moms = ih.ih_moment_images(gpu(q))
    cen, it = ih.ih_camshift(moms, gpu(starts), wh, ww, delta, max_iter)
    ocen, oit = oracle.camshift(q, starts, wh, ww, delta, max_iter)
    assert np.array_equal(it.cpu().numpy(), oit)
    assert np.array_equal(cen.cpu().numpy(), ocen)


def test_camshift_degenerate_and_errors():
    ih = ihlib()
    q = np.zeros((40, 50), np.uint8)
    moms = ih.ih_moment_images(gpu(q))
    starts = gpu(np.array([[5.5, 6.25], [39.0, 49.0]]))
    cen, it = ih.ih_camshift(moms, starts, 5, 5)
    assert cen.cpu().numpy().tolist() == [[5.5, 6.25], [39.0, 49.0]] and it.cpu().numpy().tolist() == [1, 1]
    cen, it = ih.ih_camshift(moms, starts, 5, 5, max_iter=0)
    assert it.cpu().numpy().tolist() == [0, 0]
    with pytest.raises(ih.IHError):
        ih.ih_camshift(moms, starts, 41, 5)                       # taller than the image
    big = ih.ih_moment_images(gpu(np.zeros((800, 800), np.uint8)))
    with pytest.raises(ih.IHError, match="32-bit"):
        ih.ih_camshift(big, starts, 400, 400)                     # 255 w h (h-1) / 2 >= 2^32
    empty = torch.empty((0, 2), dtype=torch.float64, device=DEV)
    c0, i0 = ih.ih_camshift(moms, empty, 5, 5)
    assert c0.shape == (0, 2) and i0.shape == (0,)


def test_tracking_frame_pipeline():
    """Frame 0 of the 1280x720 tracking video: likelihood from the target box
    (foreground) and the box grown by its own size on every side
    (background), then CAMSHIFT from 4,096 starts scattered around the
    target, against the oracle end to end."""
    ih = ihlib()
    v = config5(n_frames=1)
    rgb = v.rgb(0)
    r, c, h, w = v.target_box(0)
    H, W = rgb.shape[1:]
    fg = (r, c, r + h, c + w)
    bg = (max(0, r - h), max(0, c - w), min(H, r + 2 * h), min(W, c + 2 * w))
    say("tracking frame", fg, bg)
    q, L = ih.ih_color_likelihood(gpu(rgb), fg, bg)
    oq, _ = oracle.color_likelihood(rgb, fg, bg)
    assert np.array_equal(q.cpu().numpy(), oq)
    rng = np.random.default_rng(5)
    starts = np.stack([r + h / 2 + rng.uniform(-h, h, 4096), c + w / 2 + rng.uniform(-w, w, 4096)], 1)
    moms = ih.ih_moment_images(q)
    cen, it = ih.ih_camshift(moms, gpu(starts), h, w, 0.5, 20)
    ocen, oit = oracle.camshift(oq, starts, h, w, 0.5, 20)
    assert np.array_equal(it.cpu().numpy(), oit)
    assert np.array_equal(cen.cpu().numpy(), ocen)
    # most starts near the target settle within a few pixels of its centre
    d = np.hypot(ocen[:, 0] - (r + h / 2), ocen[:, 1] - (c + w / 2))
    assert np.median(d) < 0.25 * max(h, w)
