"""Seeded synthetic video for the tracking workload.

Textured ellipses (diameters 20-80 px) move with random-walk velocities
(at most ``vmax`` px per frame per axis, reflected at the frame borders) over a
static textured background; slowly drifting bars pass over them and occlude
them.  Object 0 is the target.  Frames are rendered on demand, so a long
sequence costs no memory until it is used.  Like the rest of this package it
holds none of the method's arithmetic: only pixel values and coordinates.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import rgb_features, smooth


@dataclass
class Ellipse:
    ry: int                  # semi-axes, px
    rx: int
    tex: np.ndarray          # 3 x (2ry+1) x (2rx+1) uint8
    mask: np.ndarray         # (2ry+1) x (2rx+1) bool
    centers: np.ndarray      # n_frames x 2 int (row, column)


@dataclass
class Bar:
    vertical: bool
    pos: np.ndarray          # n_frames, first row / column of the bar
    width: int
    color: np.ndarray        # 3 uint8


class Video:
    def __init__(self, seed: int, H: int = 720, W: int = 1280, n_frames: int = 300,
                 n_objects: Optional[int] = None, vmax: float = 8.0, accel: float = 1.5,
                 n_bars: int = 2, margin: int = 40):
        rng = np.random.default_rng(seed)
        self.H, self.W, self.n_frames = H, W, n_frames
        bg = []
        for _ in range(3):
            f = 0.5 * smooth(rng, H, W, 64) + 0.3 * smooth(rng, H, W, 16) + 0.2 * smooth(rng, H, W, 4)
            bg.append(np.clip(255.0 * f, 0, 255).astype(np.uint8))
        self.background = np.stack(bg)
        if n_objects is None:
            n_objects = int(rng.integers(1, 5))
        self.objects: List[Ellipse] = []
        for _ in range(n_objects):
            ry, rx = (int(v) for v in rng.integers(10, 41, size=2))
            h, w = 2 * ry + 1, 2 * rx + 1
            yy, xx = np.mgrid[-ry:ry + 1, -rx:rx + 1]
            mask = (yy / (ry + 0.5)) ** 2 + (xx / (rx + 0.5)) ** 2 <= 1.0
            base = rng.integers(30, 226, size=3)
            tex = np.stack([base[c] + 90.0 * (smooth(rng, h, w, 6) - 0.5) + 40.0 * (smooth(rng, h, w, 2) - 0.5)
                            for c in range(3)])
            tex = np.clip(tex, 0, 255).astype(np.uint8)
            lo = np.array([margin + ry, margin + rx], np.float64)
            hi = np.array([H - 1 - margin - ry, W - 1 - margin - rx], np.float64)
            p = lo + rng.random(2) * (hi - lo)
            v = (rng.random(2) - 0.5) * vmax
            cs = np.empty((n_frames, 2), np.int64)
            for t in range(n_frames):
                cs[t] = np.rint(p)
                v = np.clip(v + rng.normal(0.0, accel, 2), -vmax, vmax)
                p = p + v
                for a in range(2):
                    if p[a] < lo[a]:
                        p[a], v[a] = 2 * lo[a] - p[a], -v[a]
                    elif p[a] > hi[a]:
                        p[a], v[a] = 2 * hi[a] - p[a], -v[a]
                    p[a] = min(max(p[a], lo[a]), hi[a])
            self.objects.append(Ellipse(ry, rx, tex, mask, cs))
        self.bars: List[Bar] = []
        for _ in range(n_bars):
            vertical = bool(rng.integers(0, 2))
            extent = W if vertical else H
            width = int(rng.integers(6, 15))
            start = rng.random() * extent
            speed = (0.5 + 1.5 * rng.random()) * (1 if rng.integers(0, 2) else -1)
            pos = np.mod(np.rint(start + speed * np.arange(n_frames)), extent).astype(np.int64)
            self.bars.append(Bar(vertical, pos, width, rng.integers(0, 256, size=3).astype(np.uint8)))

    # ------------------------------------------------------------------ #
    def rgb(self, t: int) -> np.ndarray:
        """Frame t as 3 x H x W uint8."""
        img = self.background.copy()
        for o in self.objects:
            r, c = o.centers[t]
            r0, c0 = r - o.ry, c - o.rx
            sub = img[:, r0:r0 + o.mask.shape[0], c0:c0 + o.mask.shape[1]]
            sub[:, o.mask] = o.tex[:, o.mask]
        for b in self.bars:
            p = int(b.pos[t])
            if b.vertical:
                img[:, :, p:p + b.width] = b.color[:, None, None]
            else:
                img[:, p:p + b.width, :] = b.color[:, None, None]
        return img

    def features(self, t: int) -> np.ndarray:
        """Frame t as the seven uint8 feature channels (7 x H x W)."""
        return rgb_features(*self.rgb(t))

    def target_box(self, t: int):
        """(row, column, height, width) of the target's bounding box in frame t."""
        o = self.objects[0]
        r, c = o.centers[t]
        return int(r - o.ry), int(c - o.rx), 2 * o.ry + 1, 2 * o.rx + 1


def render(video: Video, frames: Optional[Sequence[int]] = None, threads: int = 8) -> np.ndarray:
    """Feature channels of the given frames (default: all), T x 7 x H x W uint8."""
    ts = list(range(video.n_frames)) if frames is None else list(frames)
    out = np.empty((len(ts), 7, video.H, video.W), np.uint8)

    def one(i):
        out[i] = video.features(ts[i])

    with ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(one, range(len(ts))))
    return out


def config5(n_frames: int = 300, seed: int = 500, H: int = 720, W: int = 1280) -> Video:
    """The learned-proposal tracking workload: 1280 x 720, 300 frames, 1-4 ellipses."""
    return Video(seed, H, W, n_frames)


def training_videos(n: int, n_frames: int, H: int = 360, W: int = 640, seed0: int = 9000) -> List[Video]:
    """Independent sequences (seeds disjoint from config5's) for training the proposal network."""
    return [Video(seed0 + i, H, W, n_frames) for i in range(n)]
