"""Seeded synthetic inputs for the integral-histogram workloads.

These generators stand in for the thesis's video datasets (VOT2016, ARGUS,
ABQ, WAMI PSS), which are not available: they draw images, rectangle lists,
window lists and candidate grids with the shapes, sizes and value structure
of the workloads the thesis times (smooth textured fields with noise, bright
vehicle-sized blobs, uneven frame sizes).  Everything is seeded
``numpy.random.default_rng``.

This module holds none of the method's arithmetic (no binning, no scans, no
histograms): it only produces raw pixel values and coordinates, and it serves
both the CPU oracle and the GPU path.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def smooth(rng: np.random.Generator, H: int, W: int, cell: int, dtype=np.float32) -> np.ndarray:
    """Bilinear upsampling of a uniform [0,1) lattice with spacing ``cell`` px."""
    gh, gw = H // cell + 2, W // cell + 2
    lat = rng.random((gh, gw)).astype(np.float32)
    ys = np.arange(H, dtype=np.float64) / cell
    xs = np.arange(W, dtype=np.float64) / cell
    y0 = np.floor(ys).astype(np.int64)
    x0 = np.floor(xs).astype(np.int64)
    fy = (ys - y0).astype(np.float32)[:, None]
    fx = (xs - x0).astype(np.float32)[None, :]
    # separable: along columns for every lattice row, then along rows
    across = lat[:, x0] * (1 - fx) + lat[:, x0 + 1] * fx          # gh x W
    out = np.empty((H, W), dtype)
    step = max(1, (1 << 22) // max(W, 1))
    for a in range(0, H, step):
        b = min(H, a + step)
        yy = y0[a:b]
        f = fy[a:b]
        out[a:b] = across[yy] * (1 - f) + across[yy + 1] * f
    return out


def gray_u8(seed: int, H: int, W: int) -> np.ndarray:
    """Smooth seeded field plus uniform noise, clipped to uint8."""
    rng = np.random.default_rng(seed)
    f = 200.0 * smooth(rng, H, W, 32) + rng.integers(0, 56, size=(H, W))
    return np.clip(f, 0, 255).astype(np.uint8)


def rects_uniform(seed: int, H: int, W: int, n: int, lo: int, hi: int) -> np.ndarray:
    """n half-open rectangles {r0, c0, r1, c1}; sides ~ U{lo..hi}, uniform placement."""
    rng = np.random.default_rng(seed)
    h = rng.integers(lo, min(hi, H) + 1, size=n)
    w = rng.integers(lo, min(hi, W) + 1, size=n)
    r0 = (rng.random(n) * (H - h + 1)).astype(np.int64)
    c0 = (rng.random(n) * (W - w + 1)).astype(np.int64)
    return np.stack([r0, c0, r0 + h, c0 + w], axis=1).astype(np.int32)


def _sobel(I: np.ndarray):
    p = np.pad(I.astype(np.float64), 1, mode="edge")
    gx = (p[:-2, 2:] + 2 * p[1:-1, 2:] + p[2:, 2:]) - (p[:-2, :-2] + 2 * p[1:-1, :-2] + p[2:, :-2])
    gy = (p[2:, :-2] + 2 * p[2:, 1:-1] + p[2:, 2:]) - (p[:-2, :-2] + 2 * p[:-2, 1:-1] + p[:-2, 2:])
    return gx, gy


def feature_channels(seed_base: int, H: int, W: int) -> np.ndarray:
    """Seven uint8 feature channels R, G, B, I, GO, GM, Edge (C x H x W).

    R, G, B are multi-scale textured noise; intensity is their rounded mean;
    gradient orientation, magnitude and a binary edge map come from a 3x3
    Sobel filter on the intensity with replicated borders.
    """
    chans = []
    for k in range(3):
        rng = np.random.default_rng(seed_base + k)
        f = 0.5 * smooth(rng, H, W, 64) + 0.3 * smooth(rng, H, W, 16) + 0.2 * smooth(rng, H, W, 4)
        chans.append(np.clip(255.0 * f, 0, 255).astype(np.uint8))
    return rgb_features(*chans)


def rgb_features(R: np.ndarray, G: np.ndarray, B: np.ndarray) -> np.ndarray:
    """The seven uint8 channels R, G, B, I, GO, GM, Edge of an RGB image: the
    intensity is the rounded mean; orientation, magnitude and a binary edge
    map (top 20% of magnitudes) come from a 3x3 Sobel filter on the intensity
    with replicated borders."""
    I = np.rint((R.astype(np.float64) + G + B) / 3.0).astype(np.uint8)
    gx, gy = _sobel(I)
    mag = np.sqrt(gx * gx + gy * gy)
    go = np.floor(np.mod(np.arctan2(gy, gx), np.pi) / np.pi * 256.0)
    go = np.clip(go, 0, 255).astype(np.uint8)
    gm = np.floor(255.0 * np.minimum(1.0, mag / 1443.0)).astype(np.uint8)
    edge = np.where(mag >= np.percentile(mag, 80), 255, 0).astype(np.uint8)
    return np.stack([R, G, B, I, go, gm, edge])


def aerial_u16(seed: int, H: int, W: int, n_blobs: int, blob_seed: int):
    """Multi-scale uint16 field with bright 6x12 / 12x6 blobs; returns (img, blobs)."""
    rng = np.random.default_rng(seed)
    acc = np.zeros((H, W), np.float32)
    for cell, a in zip((1024, 256, 64, 16, 4), (0.4, 0.25, 0.15, 0.1, 0.1)):
        acc += np.float32(a) * smooth(rng, H, W, min(cell, max(H, W)))
    img = np.clip(40000.0 * acc, 0, 65535).astype(np.uint16)
    del acc
    brng = np.random.default_rng(blob_seed)
    blobs = []
    margin = 16
    for _ in range(n_blobs):
        vertical = bool(brng.integers(0, 2))
        bh, bw = (12, 6) if vertical else (6, 12)
        r = int(brng.integers(margin, H - margin - bh))
        c = int(brng.integers(margin, W - margin - bw))
        img[r:r + bh, c:c + bw] = brng.integers(50000, 65536, size=(bh, bw), dtype=np.uint16)
        blobs.append((r, c, bh, bw))
    return img, np.asarray(blobs, np.int32)


def grid_origins(r0: int, c0: int, ny: int, nx: int) -> np.ndarray:
    """Row-major candidate origins (r0+dy, c0+dx), dy < ny outer, dx < nx inner."""
    dy, dx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([r0 + dy.ravel(), c0 + dx.ravel()], axis=1).astype(np.int32)


# --------------------------------------------------------------------------- #
# Workload configurations                                                     #
# --------------------------------------------------------------------------- #
@dataclass
class Workload:
    name: str
    img: np.ndarray            # C x H x W, uint8 or uint16
    bins: int
    bits: int
    rects: Optional[np.ndarray] = None      # plain queries {r0,c0,r1,c1}
    windows: Optional[np.ndarray] = None    # weighted queries {r0,c0,r1,c1}
    tmpl_win: Optional[tuple] = None        # template window (r, c, h, w)
    origins: Optional[np.ndarray] = None    # candidate origins (n x 2)
    moments: bool = False
    extra: dict = field(default_factory=dict)

    @property
    def C(self):
        return self.img.shape[0]

    @property
    def H(self):
        return self.img.shape[1]

    @property
    def W(self):
        return self.img.shape[2]

    @property
    def P(self):
        return self.C * self.bins


def config1(scale: float = 1.0, n_rects: int = 10_000) -> Workload:
    """640x480 uint8 grayscale, 32 bins; 10,000 rectangles with sides 4-200 px."""
    H, W = max(8, int(480 * scale)), max(8, int(640 * scale))
    img = gray_u8(101, H, W)[None]
    rects = rects_uniform(102, H, W, n_rects, 4, 200)
    return Workload("640x480 u8 gray, 32 bins, 10k rect queries", img, 32, 8, rects=rects)


def config2(scale: float = 1.0, n_windows: int = 100_000) -> Workload:
    """1920x1080, 7 u8 feature channels x 16 bins (112 planes); SWIH windows 16-256 px."""
    H, W = max(16, int(1080 * scale)), max(16, int(1920 * scale))
    img = feature_channels(201, H, W)
    wins = rects_uniform(204, H, W, n_windows, 16, 256)
    return Workload("1920x1080 7ch u8, 7x16 bins + moments, 100k weighted queries", img, 16, 8,
                    windows=wins, moments=True)


def phog_inputs(scale: float = 1.0, seed_base: int = 201):
    """Inputs of the magnitude-weighted orientation histogram at 1920x1080 (the
    config-2 scene): gradient orientation (the binned image), gradient
    magnitude (the weight) and the binary edge map (the mask), each 1 x H x W
    uint8."""
    H, W = max(16, int(1080 * scale)), max(16, int(1920 * scale))
    f = feature_channels(seed_base, H, W)
    return f[4:5].copy(), f[5:6].copy(), f[6:7].copy()


def surveillance_video(seed: int, n_frames: int, H: int = 576, W: int = 768, n_movers: int = 12,
                       noise: int = 6) -> np.ndarray:
    """Grey surveillance-style video (n_frames x H x W uint8), the input of the
    spatio-temporal median: a static textured background (200 smooth(cell 32)
    + 40 smooth(cell 4)), n_movers rectangles 8-60 px a side with their own
    grey level U{0..255} moving at a constant velocity of 0.5-4 px/frame
    (reflected at the borders), and fresh per-frame noise U{-noise..noise}."""
    rng = np.random.default_rng(seed)
    bg = 200.0 * smooth(rng, H, W, 32) + 40.0 * smooth(rng, H, W, 4)
    hs = rng.integers(8, 61, n_movers)
    ws = rng.integers(8, 61, n_movers)
    y = rng.uniform(0, H - hs)
    x = rng.uniform(0, W - ws)
    speed = rng.uniform(0.5, 4.0, n_movers)
    ang = rng.uniform(0, 2 * np.pi, n_movers)
    vy, vx = speed * np.sin(ang), speed * np.cos(ang)
    level = rng.integers(0, 256, n_movers)
    out = np.empty((n_frames, H, W), np.uint8)
    for f in range(n_frames):
        img = bg.copy()
        for i in range(n_movers):
            r0, c0 = int(y[i]), int(x[i])
            img[r0:r0 + hs[i], c0:c0 + ws[i]] = level[i]
        img += rng.integers(-noise, noise + 1, size=(H, W))
        out[f] = np.clip(img, 0, 255).astype(np.uint8)
        y += vy
        x += vx
        for i in range(n_movers):
            if y[i] < 0 or y[i] > H - hs[i]:
                vy[i] = -vy[i]
                y[i] = min(max(y[i], 0), H - hs[i])
            if x[i] < 0 or x[i] > W - ws[i]:
                vx[i] = -vx[i]
                x[i] = min(max(x[i], 0), W - ws[i])
    return out


def config3(scale: float = 1.0, n_rects: int = 1_000_000, n_blobs: int = 2000,
            radius: int = 64, shifted: bool = False) -> Workload:
    """8192^2 uint16 aerial-style frame, 64 bins; 1M rects; 129x129 candidate grid."""
    S = max(256, int(8192 * scale))
    img, blobs = aerial_u16(301, S, S, max(1, int(n_blobs * scale * scale)), 302)
    rects = rects_uniform(303, S, S, n_rects, 4, 200)
    # template: the 32x32 window centred on blob 0, kept inside the frame
    br, bc, bh, bw = (int(v) for v in blobs[0])
    tr = min(max(br + bh // 2 - 16, radius), S - 32 - radius)
    tc = min(max(bc + bw // 2 - 16, radius), S - 32 - radius)
    frame = img
    if shifted:
        rng = np.random.default_rng(304)
        dy, dx = (int(v) for v in rng.integers(-40, 41, size=2))
        frame = np.roll(img, (dy, dx), axis=(0, 1))
        noise = rng.integers(0, 1024, size=frame.shape, dtype=np.uint16)
        frame = np.minimum(frame.astype(np.uint32) + noise, 65535).astype(np.uint16)
    origins = grid_origins(tr - radius, tc - radius, 2 * radius + 1, 2 * radius + 1)
    return Workload("8192x8192 u16, 64 bins, 1M rects, 129x129 pyramid chi2 match", frame[None], 64, 16,
                    rects=rects, tmpl_win=(tr, tc, 32, 32), origins=origins,
                    extra={"template_img": img[None], "blobs": blobs})


@dataclass
class Frame:
    img: np.ndarray
    bins: int
    bits: int
    tmpl_win: tuple
    origins: np.ndarray


def config4(n_frames: int = 64, scale: float = 1.0, grid: int = 64) -> List[Frame]:
    """64 uint8 frames of uneven size (320x240 .. 2048x2048), bins from {8,16,32,64};
    per frame a 32x32 template and a grid x grid set of candidate origins around it."""
    frames = []
    for f in range(n_frames):
        rng = np.random.default_rng(400 + f)
        W = max(48 + grid, int(rng.integers(320, 2049) * scale))
        H = max(48 + grid, int(rng.integers(240, 2049) * scale))
        bins = int(rng.choice([8, 16, 32, 64]))
        img = gray_u8(1400 + f, H, W)[None]
        half = grid // 2
        tr = int(rng.integers(half, H - 32 - half + 1))
        tc = int(rng.integers(half, W - 32 - half + 1))
        origins = grid_origins(tr - half, tc - half, grid, grid)
        frames.append(Frame(img, bins, 8, (tr, tc, 32, 32), origins))
    return frames
