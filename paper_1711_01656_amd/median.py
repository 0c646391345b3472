"""Spatio-temporal median background model (Alg. 4, Sec. 4.1.1) on the GPU.

Frames are pushed one at a time.  The last T+1 frames stay on the device in a
ring; the joint integral histogram (JIH) of that window is updated in place by
``ih_jih_update`` (the entering frame counted in, the leaving one counted out)
and, once the window is full, every push yields the median bin of each
pixel's win_h x win_w x (T+1) box for the window's centre frame
(``ih_local_median``).  Every step runs in the library's kernels; this module
only keeps the ring and the frame count.
"""
from __future__ import annotations

from typing import Optional, Tuple

import torch

from . import ih


class SpatioTemporalMedian:
    def __init__(self, C: int, H: int, W: int, bins: int, T: int, win_h: int = 1, win_w: int = 1,
                 dtype: torch.dtype = torch.uint8, value_bits: Optional[int] = None, layout: str = "bhw",
                 device="cuda:0", cfg: Optional[ih.TileCfg] = None):
        if T < 0:
            raise ih.IHError("T must be >= 0")
        self.C, self.H, self.W, self.bins, self.T = C, H, W, bins, T
        self.win_h, self.win_w, self.layout, self.cfg = win_h, win_w, layout, cfg
        self.value_bits = value_bits
        P = C * bins
        self.ring = torch.empty((T + 1, C, H, W), dtype=dtype, device=device)
        self.jih = torch.zeros(ih.shape_of(P, H, W, layout), dtype=torch.int32, device=device)
        self.ws = torch.empty(ih.jih_update_workspace_size(H, W, C, bins, cfg, layout), dtype=torch.uint8,
                              device=device)
        self.median = torch.empty((C, H, W), dtype=torch.int32, device=device)
        self.count = 0

    @property
    def frames(self) -> int:
        """Frames currently in the window."""
        return min(self.count, self.T + 1)

    def push(self, frame: torch.Tensor) -> Optional[Tuple[int, torch.Tensor]]:
        """Add the next frame (C x H x W, or H x W for one channel).  Returns
        (index of the centre frame, C x H x W median bins) once T+1 frames have
        been pushed, else None.  The returned tensor is overwritten by the
        next push."""
        if frame.dim() == 2:
            frame = frame.unsqueeze(0)
        slot = self.count % (self.T + 1)
        tail = self.ring[slot] if self.count > self.T else None
        ih.ih_jih_update(frame, tail, self.bins, self.jih, self.value_bits, self.cfg, self.ws, self.layout)
        self.ring[slot].copy_(frame)
        self.count += 1
        if self.count <= self.T:
            return None
        ih.ih_local_median(self.jih, self.C, self.bins, self.T + 1, self.win_h, self.win_w, out=self.median,
                           layout=self.layout)
        return self.count - 1 - self.T // 2, self.median
