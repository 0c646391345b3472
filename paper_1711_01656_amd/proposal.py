"""Learned candidate proposal: binding of the ``ih_lp_*`` C ABI (include/ih_lp.h).

A small BF16 convolutional network scores the 65 x 65 candidate offsets of
the tracker's search region from a 7 x 128 x 128 crop of the feature channels
centred on the previous target position.  Every step of inference and training
(crop, convolutions, head, loss, gradients, SGD, top-k) runs in libih.so's
gfx950 kernels; this module allocates buffers and sequences the calls.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional

import numpy as np
import torch

from .ih import IHError, _check, _dev, _p, lib

C_IN, C_MID, CROP, SMAP, RADIUS = 7, 32, 128, 64, 32
NOFF = 2 * RADIUS + 1                 # offsets per axis
N_OFFSETS = NOFF * NOFF               # 4225
# (name, shape) of the FP32 parameter array, in order
PARAM_LAYOUT = (("W1", (C_MID, C_IN, 3, 3)), ("b1", (C_MID,)),
                ("W2", (C_MID, C_MID, 3, 3)), ("b2", (C_MID,)),
                ("W3", (C_MID, C_MID, 3, 3)), ("b3", (C_MID,)),
                ("wh", (C_MID,)), ("bh", (1,)))
# (Cin, stride, dilation, pad) of the three convolutions; receptive field
# 3 + 2*3*2 + 2*9*2 = 51 input pixels, wide enough to see the outline of
# targets up to about 50 px from their centre
LAYERS = ((C_IN, 2, 1, 1), (C_MID, 1, 3, 3), (C_MID, 1, 9, 9))
def wgrad_chunk(npix: int) -> int:
    """Pixels per weight-gradient partial sum: at least 1024, and at most
    about 64 partial rows to add (the summation order depends only on npix)."""
    per = -(-npix // 64)
    return max(1024, (per + 7) // 8 * 8)


def _offsets():
    off, o = {}, 0
    for name, shape in PARAM_LAYOUT:
        n = int(np.prod(shape))
        off[name] = (o, n, shape)
        o += n
    return off, o


PARAM_OFFSETS, N_PARAMS = _offsets()


def label_of(dy, dx):
    """Flat logit index of offset (dy, dx), each in [-32, 32]."""
    return (np.asarray(dy) + RADIUS) * NOFF + (np.asarray(dx) + RADIUS)


def offset_of(idx):
    """(dy, dx) of flat logit indices."""
    idx = np.asarray(idx)
    return idx // NOFF - RADIUS, idx % NOFF - RADIUS


def _s(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


# ------------------------------------------------------------ thin calls --
def lp_crop(feat: torch.Tensor, centers: torch.Tensor, x: torch.Tensor, side: int = CROP,
            frames: Optional[torch.Tensor] = None):
    """Crops of feat (C x H x W, or F x C x H x W with a frame index per crop)."""
    _dev(feat, "feat", torch.uint8)
    _dev(centers, "centers", torch.int32)
    _dev(x, "x", torch.bfloat16)
    if feat.dim() == 3:
        feat = feat.unsqueeze(0)
    F, C, H, W = feat.shape
    B = centers.shape[0]
    if centers.shape != (B, 2) or x.numel() != B * C * side * side:
        raise IHError("centers must be B x 2 and x must hold B x C x side x side values")
    if frames is not None:
        _dev(frames, "frames", torch.int32)
        if frames.numel() != B:
            raise IHError("frames must hold one index per crop")
    _check(lib().ih_lp_crop(_p(feat), F, C, H, W, _p(frames), _p(centers), B, side, _p(x), _s(x)), "ih_lp_crop")


def lp_origins(base: torch.Tensor, radius: int = RADIUS, idx: Optional[torch.Tensor] = None,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Candidate origins base + offset for the offsets idx (B x k) or all of them."""
    _dev(base, "base", torch.int32)
    B = base.shape[0]
    n = (2 * radius + 1) ** 2
    if idx is not None:
        _dev(idx, "idx", torch.int32)
        k = idx.numel() // B
    else:
        k = n
    if out is None:
        out = torch.empty((B * k, 2), dtype=torch.int32, device=base.device)
    _dev(out, "origins", torch.int32)
    if out.numel() != B * k * 2 or base.numel() != 2 * B:
        raise IHError("lp_origins: shape mismatch")
    _check(lib().ih_lp_origins(_p(idx), B, k, _p(base), radius, _p(out), _s(out)), "ih_lp_origins")
    return out


def lp_conv(inp: torch.Tensor, w: torch.Tensor, bias: Optional[torch.Tensor], stride: int, dil: int, pad: int,
            out: torch.Tensor, mask: Optional[torch.Tensor] = None):
    _dev(inp, "in", torch.bfloat16)
    _dev(w, "w", torch.bfloat16)
    _dev(out, "out", torch.bfloat16)
    B, Cin, Hin, Win = inp.shape
    Ho = (Hin + 2 * pad - 2 * dil - 1) // stride + 1
    Wo = (Win + 2 * pad - 2 * dil - 1) // stride + 1
    kt = 9 * ((Cin + 7) // 8 * 8)
    if tuple(out.shape) != (B, C_MID, Ho, Wo) or w.numel() != C_MID * kt:
        raise IHError("lp_conv: output or weight shape mismatch")
    if mask is not None:
        _dev(mask, "mask", torch.bfloat16)
        if mask.shape != out.shape:
            raise IHError("lp_conv: mask shape mismatch")
    elif bias is None:
        raise IHError("lp_conv: forward needs a bias")
    else:
        _dev(bias, "bias", torch.float32)
    _check(lib().ih_lp_conv(_p(inp), B, Cin, Hin, Win, _p(w), _p(bias), stride, dil, pad, _p(mask), _p(out),
                            _s(out)), "ih_lp_conv")


def lp_wgrad(inp: torch.Tensor, dz: torch.Tensor, stride: int, dil: int, pad: int, dw: torch.Tensor,
             db: torch.Tensor, ws: Optional[torch.Tensor] = None, chunk: Optional[int] = None):
    _dev(inp, "in", torch.bfloat16)
    _dev(dz, "dz", torch.bfloat16)
    _dev(dw, "dw", torch.float32)
    _dev(db, "db", torch.float32)
    B, Cin, Hin, Win = inp.shape
    if chunk is None:
        chunk = wgrad_chunk(dz.numel() // C_MID)
    need = lib().ih_lp_wgrad_workspace(B, Cin, Hin, Win, stride, dil, pad, chunk)
    if need == 0:
        raise IHError("lp_wgrad: invalid shape")
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need // 4, dtype=torch.float32, device=inp.device)
    if dw.numel() != C_MID * Cin * 9 or db.numel() != C_MID or dz.shape[:2] != (B, C_MID):
        raise IHError("lp_wgrad: gradient shape mismatch")
    _check(lib().ih_lp_wgrad(_p(inp), _p(dz), B, Cin, Hin, Win, stride, dil, pad, chunk, _p(ws),
                             ws.numel() * ws.element_size(), _p(dw), _p(db), _s(dw)), "ih_lp_wgrad")


def lp_head(a3: torch.Tensor, wh: torch.Tensor, bh: torch.Tensor, logits: torch.Tensor):
    B = a3.shape[0]
    _dev(a3, "a3", torch.bfloat16)
    _dev(wh, "wh", torch.float32)
    _dev(bh, "bh", torch.float32)
    if wh.numel() != C_MID or bh.numel() != 1:
        raise IHError("lp_head: wh must hold 32 values and bh 1")
    _dev(logits, "logits", torch.float32)
    if tuple(a3.shape) != (B, C_MID, SMAP, SMAP) or logits.numel() != B * N_OFFSETS:
        raise IHError("lp_head: shape mismatch")
    _check(lib().ih_lp_head(_p(a3), _p(wh), _p(bh), B, _p(logits), _s(logits)), "ih_lp_head")


def lp_softmax_ce(logits: torch.Tensor, labels: torch.Tensor, loss: torch.Tensor, dlogits: torch.Tensor):
    B = labels.numel()
    _dev(labels, "labels", torch.int32)
    for t, n in ((logits, "logits"), (loss, "loss"), (dlogits, "dlogits")):
        _dev(t, n, torch.float32)
    if logits.numel() != B * N_OFFSETS or dlogits.numel() != B * N_OFFSETS or loss.numel() != B:
        raise IHError("lp_softmax_ce: shape mismatch")
    _check(lib().ih_lp_softmax_ce(_p(logits), _p(labels), B, _p(loss), _p(dlogits), _s(loss)), "ih_lp_softmax_ce")


def lp_head_bwd(dlogits, a3, wh, ds, dz3, dwh, dbh, ws: Optional[torch.Tensor] = None):
    B = a3.shape[0]
    for t, n in ((dlogits, "dlogits"), (wh, "wh"), (ds, "ds"), (dwh, "dwh"), (dbh, "dbh")):
        _dev(t, n, torch.float32)
    _dev(a3, "a3", torch.bfloat16)
    if tuple(a3.shape) != (B, C_MID, SMAP, SMAP) or dlogits.numel() != B * N_OFFSETS or wh.numel() != C_MID:
        raise IHError("lp_head_bwd: shape mismatch")
    if ds.numel() != B * SMAP * SMAP or dz3.shape != a3.shape or dwh.numel() != C_MID or dbh.numel() != 1:
        raise IHError("lp_head_bwd: shape mismatch")
    _dev(dz3, "dz3", torch.bfloat16)
    if ws is None or ws.numel() < B * (C_MID + 1):
        ws = torch.empty(B * (C_MID + 1), dtype=torch.float32, device=a3.device)
    _dev(ws, "ws", torch.float32)
    _check(lib().ih_lp_head_bwd(_p(dlogits), _p(a3), _p(wh), B, _p(ds), _p(dz3), _p(dwh), _p(dbh), _p(ws), _s(ds)),
           "ih_lp_head_bwd")


def lp_pack(params: torch.Tensor, w1, w2, w3, w2t, w3t):
    _dev(params, "params", torch.float32)
    if params.numel() != N_PARAMS:
        raise IHError("lp_pack: params must hold %d floats" % N_PARAMS)
    for t, n, name in ((w1, C_MID * 72, "w1"), (w2, C_MID * 288, "w2"), (w3, C_MID * 288, "w3"),
                       (w2t, C_MID * 288, "w2t"), (w3t, C_MID * 288, "w3t")):
        _dev(t, name, torch.bfloat16)
        if t.numel() != n:
            raise IHError("lp_pack: %s must hold %d values" % (name, n))
    _check(lib().ih_lp_pack(_p(params), _p(w1), _p(w2), _p(w3), _p(w2t), _p(w3t), _s(params)), "ih_lp_pack")


def lp_sgd(params: torch.Tensor, grads: torch.Tensor, mom: torch.Tensor, lr: float, momentum: float,
           weight_decay: float):
    for t, n in ((params, "params"), (grads, "grads"), (mom, "mom")):
        _dev(t, n, torch.float32)
    if not (params.numel() == grads.numel() == mom.numel()):
        raise IHError("lp_sgd: size mismatch")
    _check(lib().ih_lp_sgd(_p(params), _p(grads), _p(mom), params.numel(), lr, momentum, weight_decay,
                           _s(params)), "ih_lp_sgd")


def lp_topk(logits: torch.Tensor, k: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    _dev(logits, "logits", torch.float32)
    B = logits.shape[0]
    n = logits.numel() // B
    if out is None:
        out = torch.empty((B, k), dtype=torch.int32, device=logits.device)
    _check(lib().ih_lp_topk(_p(logits), B, n, k, _p(out), _s(logits)), "ih_lp_topk")
    return out


# ---------------------------------------------------------------- network --
def init_params(seed: int) -> Dict[str, np.ndarray]:
    """He-normal FP32 initial weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in PARAM_LAYOUT:
        if name.startswith("W"):
            fan_in = shape[1] * 9
            p[name] = (rng.standard_normal(shape) * np.sqrt(2.0 / fan_in)).astype(np.float32)
        elif name == "wh":
            p[name] = (rng.standard_normal(shape) * np.sqrt(1.0 / C_MID)).astype(np.float32)
        else:
            p[name] = np.zeros(shape, np.float32)
    return p


class ProposalNet:
    """Device-resident network: FP32 master parameters, SGD momentum, BF16
    operands, and activation / gradient buffers for batches up to max_batch."""

    def __init__(self, params: Dict[str, np.ndarray], max_batch: int = 64, device="cuda"):
        self.device = torch.device(device)
        self.max_batch = max_batch
        self.params = torch.zeros(N_PARAMS, dtype=torch.float32, device=self.device)
        self.grads = torch.zeros_like(self.params)
        self.mom = torch.zeros_like(self.params)
        self.set_params(params)
        bf = dict(dtype=torch.bfloat16, device=self.device)
        self.w1 = torch.empty(C_MID * 72, **bf)
        self.w2, self.w3, self.w2t, self.w3t = (torch.empty(C_MID * 288, **bf) for _ in range(4))
        B = max_batch
        self.x = torch.empty((B, C_IN, CROP, CROP), **bf)
        self.a = [None] + [torch.empty((B, C_MID, SMAP, SMAP), **bf) for _ in range(3)]
        self.dz = [None] + [torch.empty((B, C_MID, SMAP, SMAP), **bf) for _ in range(3)]
        f32 = dict(dtype=torch.float32, device=self.device)
        self.logits = torch.empty((B, NOFF, NOFF), **f32)
        self.dlogits = torch.empty((B, NOFF, NOFF), **f32)
        self.loss = torch.empty(B, **f32)
        self.ds = torch.empty((B, SMAP, SMAP), **f32)
        self.labels = torch.empty(B, dtype=torch.int32, device=self.device)
        ws = max(lib().ih_lp_wgrad_workspace(b, cin, SMAP * st, SMAP * st, st, d, pd, wgrad_chunk(b * SMAP * SMAP))
                 for cin, st, d, pd in LAYERS for b in range(1, B + 1))
        self.ws = torch.empty(ws // 4, **f32)
        self.ws_head = torch.empty(B * (C_MID + 1), **f32)
        self.packed = False

    # parameters ------------------------------------------------------------
    def view(self, name: str, t: Optional[torch.Tensor] = None) -> torch.Tensor:
        o, n, shape = PARAM_OFFSETS[name]
        return (self.params if t is None else t)[o:o + n]

    def set_params(self, params: Dict[str, np.ndarray]):
        flat = np.concatenate([np.asarray(params[name], np.float32).reshape(-1) for name, _ in PARAM_LAYOUT])
        self.params.copy_(torch.from_numpy(flat))
        self.mom.zero_()
        self.packed = False

    def get_params(self, t: Optional[torch.Tensor] = None) -> Dict[str, np.ndarray]:
        flat = (self.params if t is None else t).cpu().numpy()
        return {name: flat[o:o + n].reshape(shape).copy() for name, (o, n, shape) in PARAM_OFFSETS.items()}

    def state(self) -> Dict[str, np.ndarray]:
        """Parameters and momentum as host arrays (for checkpoints)."""
        return {"params": self.params.cpu().numpy().copy(), "mom": self.mom.cpu().numpy().copy()}

    def load_state(self, st: Dict[str, np.ndarray]):
        self.params.copy_(torch.from_numpy(np.asarray(st["params"], np.float32)))
        self.mom.copy_(torch.from_numpy(np.asarray(st["mom"], np.float32)))
        self.packed = False

    def pack(self):
        lp_pack(self.params, self.w1, self.w2, self.w3, self.w2t, self.w3t)
        self.packed = True

    # passes ----------------------------------------------------------------
    def crop(self, feat: torch.Tensor, centers: torch.Tensor, frames: Optional[torch.Tensor] = None):
        """Network inputs for crops of feat (C x H x W u8, or F x C x H x W with
        frame indices) centred at centers (B x 2)."""
        B = centers.shape[0]
        self._check_batch(B)
        x = self.x[:B]
        lp_crop(feat, centers, x, frames=frames)
        return x

    def _check_batch(self, B):
        if B < 1 or B > self.max_batch:
            raise IHError("batch %d outside 1..%d" % (B, self.max_batch))

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """Logits (B x 65 x 65) of the inputs x (B x 7 x 128 x 128 bf16)."""
        B = x.shape[0]
        self._check_batch(B)
        if not self.packed:
            self.pack()
        ws = (self.w1, self.w2, self.w3)
        inp = x
        for i, (cin, st, d, pd) in enumerate(LAYERS, 1):
            lp_conv(inp, ws[i - 1], self.view("b%d" % i), st, d, pd, self.a[i][:B])
            inp = self.a[i][:B]
        lp_head(inp, self.view("wh"), self.view("bh"), self.logits[:B])
        return self.logits[:B]

    def backward(self, x: torch.Tensor, labels: torch.Tensor) -> torch.Tensor:
        """Loss per sample and parameter gradients (self.grads) of the mean
        softmax cross-entropy; forward() must have run on the same x."""
        B = x.shape[0]
        lp_softmax_ce(self.logits[:B], labels, self.loss[:B], self.dlogits[:B])
        g = self.grads
        lp_head_bwd(self.dlogits[:B], self.a[3][:B], self.view("wh"), self.ds[:B], self.dz[3][:B],
                    self.view("wh", g), self.view("bh", g), self.ws_head)
        wt = {2: self.w2t, 3: self.w3t}
        for i in (3, 2, 1):
            cin, st, d, pd = LAYERS[i - 1]
            inp = x if i == 1 else self.a[i - 1][:B]
            lp_wgrad(inp, self.dz[i][:B], st, d, pd, self.view("W%d" % i, g), self.view("b%d" % i, g), self.ws)
            if i > 1:
                # input gradient of a stride-1 layer whose pad equals its dilation
                lp_conv(self.dz[i][:B], wt[i], None, 1, d, pd, self.dz[i - 1][:B], mask=self.a[i - 1][:B])
        return self.loss[:B]

    def train_step(self, x: torch.Tensor, labels: torch.Tensor, lr: float, momentum: float = 0.9,
                   weight_decay: float = 0.0) -> torch.Tensor:
        self.forward(x)
        loss = self.backward(x, labels)
        lp_sgd(self.params, self.grads, self.mom, lr, momentum, weight_decay)
        self.packed = False
        return loss

    def propose(self, feat: torch.Tensor, centers: torch.Tensor, k: int, out: Optional[torch.Tensor] = None):
        """Top-k offset indices (B x k, best first) for crops centred at centers."""
        x = self.crop(feat, centers)
        logits = self.forward(x)
        return lp_topk(logits.view(logits.shape[0], -1), k, out)
