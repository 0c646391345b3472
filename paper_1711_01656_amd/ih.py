"""Thin Python binding of libih.so (the C ABI declared in include/ih.h).

Argument marshalling only: every computation runs in the library's gfx950
kernels.  PyTorch supplies device memory and the current HIP stream.  The
functions keep the C names (``ih_build``, ``ih_query_rect``, ...).  There is
no fallback: if the library is missing or fails to load, every call raises.

Layouts: ``"bhw"`` tensors are P x H x W (bin-major, the thesis's layout);
``"hwb"`` tensors are H x W x P (planes innermost).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libih.so")
_lib = None

IH_OK = 0
IH_U8, IH_U16 = 0, 1
IH_CHI2, IH_L1, IH_PMK = 0, 1, 2
IH_MANHATTAN = 0
IH_BHW, IH_HWB = 0, 1
METRICS = {"chi2": IH_CHI2, "l1": IH_L1, "pmk": IH_PMK}
LAYOUTS = {"bhw": IH_BHW, "hwb": IH_HWB}
BATCH_MODES = {"phased": 0, "cooperative": 1}

# C declarations mirrored from include/ih.h: name -> (restype, argtypes)
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t


class Rect(ctypes.Structure):
    """A half-open rectangle [r0, r1) x [c0, c1) (ih_rect in include/ih.h)."""
    _fields_ = [("r0", ctypes.c_int32), ("c0", ctypes.c_int32), ("r1", ctypes.c_int32), ("c1", ctypes.c_int32)]


SIGNATURES = {
    "ih_version": (ctypes.c_int, []),
    "ih_last_error": (ctypes.c_char_p, []),
    "ih_build_workspace_size": (_SZ, [_I32, _I32, _I32, _I32, _I32, _I32, _P]),
    "ih_build": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _P, _SZ, _P]),
    "ih_build_noalloc": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _P, _P]),
    "ih_build_weighted": (ctypes.c_int, [_P, _I32, _P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _SZ,
                                         _P]),
    "ih_jih_update_workspace_size": (_SZ, [_I32, _I32, _I32, _I32, _I32, _P]),
    "ih_jih_update": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "ih_color_likelihood_workspace_size": (_SZ, []),
    "ih_color_likelihood": (ctypes.c_int, [_P, _I32, _I32, Rect, Rect, _P, _SZ, _P, _P, _P]),
    "ih_moment_images": (ctypes.c_int, [_P, _I32, _I32, _P, _P, _P, _P, _P, _SZ, _P]),
    "ih_camshift": (ctypes.c_int, [_P, _P, _P, _I32, _I32, _P, _I64, _I32, _I32, ctypes.c_double, _I32, _P, _P,
                                   _P]),
    "ih_build_moments2": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _SZ, _P]),
    "ih_query_quadratic": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _I32, _I32, _I32, _I32, _P, _I64, _I32, _P,
                                          _P]),
    "ih_query_wedding": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _I32, _P, _I64, _I32, _I32, ctypes.c_double,
                                        _P, _P]),
    "ih_local_median": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P]),
    "ih_query_rect": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _P, _I64, _P, _P]),
    "ih_query_weighted": (ctypes.c_int, [_P, _P, _P, _I32, _I32, _I32, _I32, _I32, _P, _I64, _I32, _I32, _P, _P]),
    "ih_pyramid_desc": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _P, _I64, _I32, _P, _P]),
    "ih_match_candidates": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _P, _I32, _I32, _I32, _P, _I64, _I32,
                                           _P, _P, _P]),
    "ih_profile_events": (ctypes.c_int, [_P, _P]),
    "ih_set_lookback_patience": (ctypes.c_int, [_I32]),
    "ih_build_passes": (ctypes.c_int, [_I32, _P]),
    "ih_batch_plan_bytes": (_SZ, [_I32]),
    "ih_batch_plan": (ctypes.c_int, [_P, _I32, _I32, _I32, _P, _SZ, ctypes.POINTER(_SZ)]),
    "ih_build_batch": (ctypes.c_int, [_P, _P, _P, _SZ, _I32, _P]),
    # learned proposal (include/ih_lp.h)
    "ih_lp_conv": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _P, _P, _I32, _I32, _I32, _P, _P, _P]),
    "ih_lp_wgrad_workspace": (_SZ, [_I32, _I32, _I32, _I32, _I32, _I32, _I32, _I64]),
    "ih_lp_wgrad": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _I64, _P, _SZ, _P, _P, _P]),
    "ih_lp_head": (ctypes.c_int, [_P, _P, _P, _I32, _P, _P]),
    "ih_lp_softmax_ce": (ctypes.c_int, [_P, _P, _I32, _P, _P, _P]),
    "ih_lp_head_bwd": (ctypes.c_int, [_P, _P, _P, _I32, _P, _P, _P, _P, _P, _P]),
    "ih_lp_crop": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _P, _P, _I32, _I32, _P, _P]),
    "ih_lp_origins": (ctypes.c_int, [_P, _I32, _I32, _P, _I32, _P, _P]),
    "ih_lp_pack": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "ih_lp_sgd": (ctypes.c_int, [_P, _P, _P, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]),
    "ih_lp_topk": (ctypes.c_int, [_P, _I32, _I32, _I32, _P, _P]),
    "ih_track_prepare": (ctypes.c_int, [_P, _I32, _I32, _P, _P, _P]),
    "ih_track_gate": (ctypes.c_int, [_P, _P, _P, _P, _I32, ctypes.c_double, _P, _P, _P]),
    "ih_track_gate_bounded": (ctypes.c_int, [_P, _P, _P, _I32, ctypes.c_double, _P, _P, _P, _P]),
    "ih_track_commit": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _P, _I32, _P]),
    "ih_track_fetch": (ctypes.c_int, [_P, _I64, _I32, _P, _P, _P]),
    "ih_track_region": (ctypes.c_int, [_P, _I32, _I32, _I32, _P, _I32, _I32, _I32, _P, _P, _P]),
    "ih_track_refine_origins": (ctypes.c_int, [_P, _P, _I32, _I32, _P, _P, _P]),
    "ih_track_refine_pick": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _I32, _P]),
}


class IHError(RuntimeError):
    pass


PASSES_DEFAULT, PASSES_ONE, PASSES_THREE = 0, 1, 3
STATUS_VALUE_RANGE, STATUS_WAIT_TIMEOUT = 1, 2


class TileCfg(ctypes.Structure):
    """Tile shape and pass count of the build (see ih_tile_cfg in include/ih.h).
    ``passes``: 0 or 3 for the three-pass build, 1 for the single-pass one."""
    _fields_ = [("tile_h", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("planes_per_wave", ctypes.c_int32), ("passes", ctypes.c_int32)]

    def __repr__(self):
        if self.passes:
            return "TileCfg(%d, %d, %d, passes=%d)" % (self.tile_h, self.tile_w, self.planes_per_wave, self.passes)
        return "TileCfg(%d, %d, %d)" % (self.tile_h, self.tile_w, self.planes_per_wave)

    def key(self):
        return (self.tile_h, self.tile_w, self.planes_per_wave, self.passes)


def onepass(tile_h: int = 0, tile_w: int = 256, planes_per_wave: int = 1) -> TileCfg:
    """Configuration of the single-pass build: bands of tile_h rows (0: the
    library's choice), tiles of tile_w columns, planes_per_wave planes per
    worker."""
    return TileCfg(tile_h, tile_w, planes_per_wave, PASSES_ONE)


def status(ws: torch.Tensor) -> int:
    """The IH_STATUS_* bits a build left in the first word of its workspace
    (synchronises with the device)."""
    return int(ws.view(torch.uint8)[:4].view(torch.int32).item()) & 0xFFFFFFFF


def build_passes(layout: str = "bhw", cfg: Optional[TileCfg] = None) -> int:
    """Passes (1 or 3) ih_build uses for this layout and configuration."""
    n = lib().ih_build_passes(_layout(layout), ctypes.byref(cfg) if cfg is not None else None)
    _check(0 if n > 0 else n, "ih_build_passes")
    return n


def set_lookback_patience(polls: int):
    """Polls of the band above before a single-pass worker publishes its own
    aggregate and looks further up (-1: always wait for the band above)."""
    _check(lib().ih_set_lookback_patience(int(polls)), "ih_set_lookback_patience")


class Frame(ctypes.Structure):
    """One frame of a batch (ih_frame in include/ih.h)."""
    _fields_ = [("img", ctypes.c_void_p), ("ih", ctypes.c_void_p),
                ("H", ctypes.c_int32), ("W", ctypes.c_int32), ("C", ctypes.c_int32),
                ("bins", ctypes.c_int32), ("value_bits", ctypes.c_int32),
                ("tile", TileCfg),
                ("tmpl_desc", ctypes.c_void_p), ("tmpl_win", ctypes.c_int32 * 4), ("tmpl_out", ctypes.c_void_p),
                ("win_h", ctypes.c_int32), ("win_w", ctypes.c_int32),
                ("origins", ctypes.c_void_p), ("n_cand", ctypes.c_int64),
                ("dist", ctypes.c_void_p), ("best", ctypes.c_void_p), ("layout", ctypes.c_int32)]


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load libih.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise IHError("libih.so not found at %s; build it with "
                          "`python -m paper_1711_01656_amd.build`" % _LIB_PATH)
        L = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != IH_OK:
        raise IHError("%s failed (%d): %s" % (what, rc, lib().ih_last_error().decode()))


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dev(t: torch.Tensor, name: str, dtype=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise IHError("%s must be a CUDA (HIP) tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise IHError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise IHError("%s must be contiguous" % name)
    return t


def _p(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _layout(layout: str) -> int:
    if layout not in LAYOUTS:
        raise IHError("layout must be 'bhw' or 'hwb'")
    return LAYOUTS[layout]


def shape_of(P: int, H: int, W: int, layout: str = "bhw"):
    return (P, H, W) if _layout(layout) == IH_BHW else (H, W, P)


def _phw(t: torch.Tensor, layout: str):
    if t.dim() != 3:
        raise IHError("integral histogram must be 3-D")
    if _layout(layout) == IH_BHW:
        P, H, W = t.shape
    else:
        H, W, P = t.shape
    return P, H, W


def version() -> int:
    return lib().ih_version()


def workspace_size(H, W, C, bins, moments=False, cfg: Optional[TileCfg] = None, layout: str = "bhw") -> int:
    n = lib().ih_build_workspace_size(H, W, C, bins, int(bool(moments)), _layout(layout),
                                      ctypes.byref(cfg) if cfg is not None else None)
    if n == 0:
        raise IHError("ih_build_workspace_size: %s" % lib().ih_last_error().decode())
    return n


def ih_build(img: torch.Tensor, bins: int, value_bits: Optional[int] = None, moments: bool = False,
             cfg: Optional[TileCfg] = None, out: Optional[torch.Tensor] = None,
             mom_out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None,
             ws: Optional[torch.Tensor] = None, layout: str = "bhw"):
    """Integral histogram of a C x H x W (or H x W) uint8/uint16 image.

    Returns ``ih`` or ``(ih, mom_x, mom_y)`` when ``moments`` (moment tensors
    are int32 views of the uint32 values stored modulo 2^32); shapes follow
    ``layout``.
    """
    _dev(img, "img")
    if img.dim() == 2:
        img = img.unsqueeze(0)
    if img.dtype == torch.uint8:
        dt, maxbits = IH_U8, 8
    elif img.dtype == torch.uint16:
        dt, maxbits = IH_U16, 16
    else:
        raise IHError("img must be uint8 or uint16")
    C, H, W = img.shape
    bits = maxbits if value_bits is None else value_bits
    P = C * bins
    dev = img.device
    shp = shape_of(P, H, W, layout)
    if out is None:
        out = torch.empty(shp, dtype=torch.int32, device=dev)
    _dev(out, "out", torch.int32)
    if out.numel() != P * H * W:
        raise IHError("out must hold P*H*W values")
    mx = my = None
    if moments:
        if mom_out is None:
            mx = torch.empty(shp, dtype=torch.int32, device=dev)
            my = torch.empty(shp, dtype=torch.int32, device=dev)
        else:
            mx, my = mom_out
        _dev(mx, "mom_x", torch.int32)
        _dev(my, "mom_y", torch.int32)
        if mx.numel() != P * H * W or my.numel() != P * H * W:
            raise IHError("moment outputs must hold P*H*W values")
    need = workspace_size(H, W, C, bins, moments, cfg, layout)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    rc = lib().ih_build(_p(img), dt, H, W, C, bins, bits, _layout(layout), _p(out), _p(mx), _p(my),
                        ctypes.byref(cfg) if cfg is not None else None, _p(ws),
                        ws.numel() * ws.element_size(), _stream(img))
    _check(rc, "ih_build")
    return (out, mx, my) if moments else out


NOALLOC_SCRATCH_BYTES = 64 << 20


def ih_build_noalloc(img: torch.Tensor, bins: int, out: torch.Tensor, value_bits: Optional[int] = None,
                     mom_out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None, cfg: Optional[TileCfg] = None,
                     status: Optional[torch.Tensor] = None, layout: str = "bhw"):
    """ih_build without a workspace (the library's per-GPU scratch array):
    the caller passes every output, and nothing is allocated.  ``status`` (a
    one-element int32 tensor, optional) receives the build's status word."""
    _dev(img, "img")
    if img.dim() == 2:
        img = img.unsqueeze(0)
    if img.dtype == torch.uint8:
        dt, maxbits = IH_U8, 8
    elif img.dtype == torch.uint16:
        dt, maxbits = IH_U16, 16
    else:
        raise IHError("img must be uint8 or uint16")
    C, H, W = img.shape
    bits = maxbits if value_bits is None else value_bits
    P = C * bins
    _dev(out, "out", torch.int32)
    if out.numel() != P * H * W:
        raise IHError("out must hold P*H*W values")
    mx = my = None
    if mom_out is not None:
        mx, my = mom_out
        _dev(mx, "mom_x", torch.int32)
        _dev(my, "mom_y", torch.int32)
        if mx.numel() != P * H * W or my.numel() != P * H * W:
            raise IHError("moment outputs must hold P*H*W values")
    if status is not None:
        _dev(status, "status", torch.int32)
        if status.numel() < 1:
            raise IHError("status must hold one value")
    rc = lib().ih_build_noalloc(_p(img), dt, H, W, C, bins, bits, _layout(layout), _p(out), _p(mx), _p(my),
                                ctypes.byref(cfg) if cfg is not None else None, _p(status), _stream(img))
    _check(rc, "ih_build_noalloc")
    return out


def ih_build_weighted(img: torch.Tensor, bins: int, weight: torch.Tensor, mask: Optional[torch.Tensor] = None,
                      value_bits: Optional[int] = None, cfg: Optional[TileCfg] = None,
                      out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                      layout: str = "bhw") -> torch.Tensor:
    """Weighted integral histogram: plane p sums ``weight`` (uint8, same shape
    as ``img``) over the pixels of bin p whose ``mask`` byte is non-zero (all
    pixels when ``mask`` is None).  Shape follows ``layout``."""
    _dev(img, "img")
    if img.dim() == 2:
        img = img.unsqueeze(0)
    if img.dtype == torch.uint8:
        dt, maxbits = IH_U8, 8
    elif img.dtype == torch.uint16:
        dt, maxbits = IH_U16, 16
    else:
        raise IHError("img must be uint8 or uint16")
    C, H, W = img.shape
    _dev(weight, "weight", torch.uint8)
    if weight.numel() != C * H * W:
        raise IHError("weight must have the image's C*H*W values")
    if mask is not None:
        _dev(mask, "mask", torch.uint8)
        if mask.numel() != C * H * W:
            raise IHError("mask must have the image's C*H*W values")
    bits = maxbits if value_bits is None else value_bits
    P = C * bins
    if out is None:
        out = torch.empty(shape_of(P, H, W, layout), dtype=torch.int32, device=img.device)
    _dev(out, "out", torch.int32)
    if out.numel() != P * H * W:
        raise IHError("out must hold P*H*W values")
    need = workspace_size(H, W, C, bins, False, cfg, layout)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=img.device)
    rc = lib().ih_build_weighted(_p(img), dt, _p(weight), _p(mask), H, W, C, bins, bits, _layout(layout), _p(out),
                                 ctypes.byref(cfg) if cfg is not None else None, _p(ws),
                                 ws.numel() * ws.element_size(), _stream(img))
    _check(rc, "ih_build_weighted")
    return out


def _frame_dtype(img: torch.Tensor):
    if img.dtype == torch.uint8:
        return IH_U8, 8
    if img.dtype == torch.uint16:
        return IH_U16, 16
    raise IHError("frames must be uint8 or uint16")


def jih_update_workspace_size(H, W, C, bins, cfg: Optional[TileCfg] = None, layout: str = "bhw") -> int:
    n = lib().ih_jih_update_workspace_size(H, W, C, bins, _layout(layout),
                                           ctypes.byref(cfg) if cfg is not None else None)
    if n == 0:
        raise IHError("ih_jih_update_workspace_size: %s" % lib().ih_last_error().decode())
    return n


def ih_jih_update(head: torch.Tensor, tail: Optional[torch.Tensor], bins: int, jih: torch.Tensor,
                  value_bits: Optional[int] = None, cfg: Optional[TileCfg] = None,
                  ws: Optional[torch.Tensor] = None, layout: str = "bhw") -> torch.Tensor:
    """Joint integral histogram update (Alg. 4): jih += IH(head) - IH(tail), in
    place (tail None while the window fills).  Returns jih."""
    _dev(head, "head")
    if head.dim() == 2:
        head = head.unsqueeze(0)
    dt, maxbits = _frame_dtype(head)
    C, H, W = head.shape
    if tail is not None:
        _dev(tail, "tail", head.dtype)
        if tail.numel() != head.numel():
            raise IHError("tail must have the head's shape")
    bits = maxbits if value_bits is None else value_bits
    _dev(jih, "jih", torch.int32)
    if jih.numel() != C * bins * H * W:
        raise IHError("jih must hold P*H*W values")
    need = jih_update_workspace_size(H, W, C, bins, cfg, layout)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=head.device)
    rc = lib().ih_jih_update(_p(head), _p(tail), dt, H, W, C, bins, bits, _layout(layout), _p(jih),
                             ctypes.byref(cfg) if cfg is not None else None, _p(ws),
                             ws.numel() * ws.element_size(), _stream(head))
    _check(rc, "ih_jih_update")
    return jih


def ih_local_median(jih: torch.Tensor, C: int, bins: int, frames: int, win_h: int, win_w: int,
                    out: Optional[torch.Tensor] = None, layout: str = "bhw") -> torch.Tensor:
    """Per-pixel median bin of each win_h x win_w x frames box of a joint
    integral histogram (Alg. 4).  C x H x W int32."""
    _dev(jih, "jih", torch.int32)
    P, H, W = _phw(jih, layout)
    if P != C * bins:
        raise IHError("jih has %d planes, expected C*bins = %d" % (P, C * bins))
    if out is None:
        out = torch.empty((C, H, W), dtype=torch.int32, device=jih.device)
    _dev(out, "out", torch.int32)
    if out.numel() != C * H * W:
        raise IHError("out must hold C*H*W values")
    _check(lib().ih_local_median(_p(jih), C, bins, H, W, _layout(layout), frames, win_h, win_w, _p(out),
                                 _stream(jih)), "ih_local_median")
    return out


KERNELS = {"manhattan": 0, "quadratic": 1, "gaussian": 2}


def ih_build_moments2(img: torch.Tensor, bins: int, value_bits: Optional[int] = None,
                      cfg: Optional[TileCfg] = None, out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None,
                      ws: Optional[torch.Tensor] = None, layout: str = "bhw"):
    """Second coordinate-moment integral histograms (row^2 and column^2 sums
    per plane, modulo 2^32, as int32 views); shapes follow ``layout``."""
    _dev(img, "img")
    if img.dim() == 2:
        img = img.unsqueeze(0)
    dt, maxbits = _frame_dtype(img)
    C, H, W = img.shape
    bits = maxbits if value_bits is None else value_bits
    P = C * bins
    shp = shape_of(P, H, W, layout)
    if out is None:
        out = (torch.empty(shp, dtype=torch.int32, device=img.device),
               torch.empty(shp, dtype=torch.int32, device=img.device))
    mxx, myy = out
    for t, name in ((mxx, "mom_xx"), (myy, "mom_yy")):
        _dev(t, name, torch.int32)
        if t.numel() != P * H * W:
            raise IHError("%s must hold P*H*W values" % name)
    need = workspace_size(H, W, C, bins, False, cfg, layout)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=img.device)
    rc = lib().ih_build_moments2(_p(img), dt, H, W, C, bins, bits, _layout(layout), _p(mxx), _p(myy),
                                 ctypes.byref(cfg) if cfg is not None else None, _p(ws),
                                 ws.numel() * ws.element_size(), _stream(img))
    _check(rc, "ih_build_moments2")
    return mxx, myy


def ih_query_quadratic(ih: torch.Tensor, mom_x: torch.Tensor, mom_y: torch.Tensor, mom_xx: torch.Tensor,
                       mom_yy: torch.Tensor, C: int, rects: torch.Tensor, l1_normalize: bool = False,
                       out: Optional[torch.Tensor] = None, layout: str = "bhw") -> torch.Tensor:
    """Quadratic-kernel (squared Euclidean distance) weighted local histograms
    in O(1) per window; n x P float32."""
    for t, name in ((ih, "ih"), (mom_x, "mom_x"), (mom_y, "mom_y"), (mom_xx, "mom_xx"), (mom_yy, "mom_yy")):
        _dev(t, name, torch.int32)
    P, H, W = _phw(ih, layout)
    _rects(rects)
    n = rects.shape[0]
    if out is None:
        out = torch.empty((n, P), dtype=torch.float32, device=ih.device)
    _dev(out, "out", torch.float32)
    _check(lib().ih_query_quadratic(_p(ih), _p(mom_x), _p(mom_y), _p(mom_xx), _p(mom_yy), P, H, W, C,
                                    _layout(layout), _p(rects), n, int(bool(l1_normalize)), _p(out),
                                    _stream(ih)), "ih_query_quadratic")
    return out


def ih_query_wedding(ih: torch.Tensor, C: int, rects: torch.Tensor, layers: int, kernel: str = "manhattan",
                     sigma: float = 0.5, out: Optional[torch.Tensor] = None, layout: str = "bhw") -> torch.Tensor:
    """Wedding-cake approximation (Eq. 3.2) of a kernel-weighted local
    histogram from the count integral histogram; n x P float32."""
    _dev(ih, "ih", torch.int32)
    P, H, W = _phw(ih, layout)
    _rects(rects)
    n = rects.shape[0]
    if kernel not in KERNELS:
        raise IHError("kernel must be one of %s" % sorted(KERNELS))
    if out is None:
        out = torch.empty((n, P), dtype=torch.float32, device=ih.device)
    _dev(out, "out", torch.float32)
    _check(lib().ih_query_wedding(_p(ih), P, H, W, C, _layout(layout), _p(rects), n, layers, KERNELS[kernel],
                                  float(sigma), _p(out), _stream(ih)), "ih_query_wedding")
    return out


def _rect(r) -> Rect:
    r0, c0, r1, c1 = (int(v) for v in r)
    return Rect(r0, c0, r1, c1)


def ih_color_likelihood(rgb: torch.Tensor, fg, bg, q: Optional[torch.Tensor] = None,
                        L: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                        want_L: bool = True):
    """FG/BG colour likelihood (Eq. 2.18-2.21) of a 3 x H x W uint8 image with
    foreground rectangle fg and background rectangle bg (minus fg), each
    (r0, c0, r1, c1).  Returns (q uint8 codes, L float32 or None)."""
    _dev(rgb, "rgb", torch.uint8)
    if rgb.dim() != 3 or rgb.shape[0] != 3:
        raise IHError("rgb must be 3 x H x W")
    _, H, W = rgb.shape
    if q is None:
        q = torch.empty((H, W), dtype=torch.uint8, device=rgb.device)
    _dev(q, "q", torch.uint8)
    if want_L and L is None:
        L = torch.empty((H, W), dtype=torch.float32, device=rgb.device)
    if L is not None:
        _dev(L, "L", torch.float32)
    need = lib().ih_color_likelihood_workspace_size()
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=rgb.device)
    _check(lib().ih_color_likelihood(_p(rgb), H, W, _rect(fg), _rect(bg), _p(ws), ws.numel() * ws.element_size(),
                                     _p(q), _p(L), _stream(rgb)), "ih_color_likelihood")
    return q, L


def ih_moment_images(q: torch.Tensor, out=None, cfg: Optional[TileCfg] = None,
                     ws: Optional[torch.Tensor] = None):
    """Moment integral images (S, Sx, Sy) of an H x W uint8 map: int32 S, and
    Sx, Sy as int32 views of values modulo 2^32."""
    _dev(q, "q", torch.uint8)
    H, W = q.shape
    if out is None:
        out = tuple(torch.empty((H, W), dtype=torch.int32, device=q.device) for _ in range(3))
    for t, name in zip(out, ("S", "Sx", "Sy")):
        _dev(t, name, torch.int32)
        if t.numel() != H * W:
            raise IHError("%s must hold H*W values" % name)
    need = workspace_size(H, W, 1, 1, True, cfg, "bhw")
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=q.device)
    _check(lib().ih_moment_images(_p(q), H, W, _p(out[0]), _p(out[1]), _p(out[2]),
                                  ctypes.byref(cfg) if cfg is not None else None, _p(ws),
                                  ws.numel() * ws.element_size(), _stream(q)), "ih_moment_images")
    return out


def ih_camshift(moments, starts: torch.Tensor, win_h: int, win_w: int, delta: float = 0.5, max_iter: int = 20,
                centers: Optional[torch.Tensor] = None, iters: Optional[torch.Tensor] = None):
    """CAMSHIFT (Alg. 1) from n start points (n x 2 float64 row, column) on the
    moment images of ih_moment_images.  Returns (centres n x 2, steps n)."""
    S, Sx, Sy = moments
    for t, name in ((S, "S"), (Sx, "Sx"), (Sy, "Sy")):
        _dev(t, name, torch.int32)
    H, W = S.shape
    _dev(starts, "starts", torch.float64)
    if starts.dim() != 2 or starts.shape[1] != 2:
        raise IHError("starts must be n x 2")
    n = starts.shape[0]
    if centers is None:
        centers = torch.empty((n, 2), dtype=torch.float64, device=S.device)
    if iters is None:
        iters = torch.empty(n, dtype=torch.int32, device=S.device)
    _dev(centers, "centers", torch.float64)
    _dev(iters, "iters", torch.int32)
    _check(lib().ih_camshift(_p(S), _p(Sx), _p(Sy), H, W, _p(starts), n, win_h, win_w, float(delta), max_iter,
                             _p(centers), _p(iters), _stream(S)), "ih_camshift")
    return centers, iters


def _rects(rects: torch.Tensor, name="rects") -> torch.Tensor:
    _dev(rects, name, torch.int32)
    if rects.dim() != 2 or rects.shape[1] != 4:
        raise IHError("%s must be n x 4 int32" % name)
    return rects


def ih_query_rect(ih: torch.Tensor, rects: torch.Tensor, out: Optional[torch.Tensor] = None,
                  layout: str = "bhw"):
    """Eq. 2.16 region histograms: n x P int32."""
    _dev(ih, "ih", torch.int32)
    P, H, W = _phw(ih, layout)
    _rects(rects)
    n = rects.shape[0]
    if out is None:
        out = torch.empty((n, P), dtype=torch.int32, device=ih.device)
    _dev(out, "out", torch.int32)
    _check(lib().ih_query_rect(_p(ih), P, H, W, _layout(layout), _p(rects), n, _p(out), _stream(ih)),
           "ih_query_rect")
    return out


def ih_query_weighted(ih: torch.Tensor, mom_x: torch.Tensor, mom_y: torch.Tensor, C: int,
                      rects: torch.Tensor, l1_normalize: bool = False,
                      out: Optional[torch.Tensor] = None, layout: str = "bhw"):
    """Manhattan-weighted local histograms (SWIH): n x P float32."""
    _dev(ih, "ih", torch.int32)
    _dev(mom_x, "mom_x", torch.int32)
    _dev(mom_y, "mom_y", torch.int32)
    P, H, W = _phw(ih, layout)
    _rects(rects)
    n = rects.shape[0]
    if out is None:
        out = torch.empty((n, P), dtype=torch.float32, device=ih.device)
    _dev(out, "out", torch.float32)
    _check(lib().ih_query_weighted(_p(ih), _p(mom_x), _p(mom_y), P, H, W, C, _layout(layout), _p(rects), n,
                                   IH_MANHATTAN, int(bool(l1_normalize)), _p(out), _stream(ih)),
           "ih_query_weighted")
    return out


def cells(levels: int) -> int:
    return sum(4 ** l for l in range(levels))


def ih_pyramid_desc(ih: torch.Tensor, wins: torch.Tensor, levels: int = 3,
                    out: Optional[torch.Tensor] = None, layout: str = "bhw"):
    """Spatial-pyramid descriptors of windows {r, c, h, w}: n x cells x P int32."""
    _dev(ih, "ih", torch.int32)
    P, H, W = _phw(ih, layout)
    _rects(wins, "wins")
    n = wins.shape[0]
    if out is None:
        out = torch.empty((n, cells(levels), P), dtype=torch.int32, device=ih.device)
    _dev(out, "out", torch.int32)
    _check(lib().ih_pyramid_desc(_p(ih), P, H, W, _layout(layout), _p(wins), n, levels, _p(out), _stream(ih)),
           "ih_pyramid_desc")
    return out


def ih_match_candidates(ih: torch.Tensor, tmpl_desc: torch.Tensor, win_h: int, win_w: int,
                        origins: torch.Tensor, levels: int = 3, metric: str = "chi2",
                        dist: Optional[torch.Tensor] = None, best: Optional[torch.Tensor] = None,
                        layout: str = "bhw"):
    """Exhaustive candidate search: (n distances float32, best index int32[1])."""
    _dev(ih, "ih", torch.int32)
    P, H, W = _phw(ih, layout)
    _dev(tmpl_desc, "tmpl_desc", torch.int32)
    _dev(origins, "origins", torch.int32)
    if origins.dim() != 2 or origins.shape[1] != 2:
        raise IHError("origins must be n x 2 int32")
    if tmpl_desc.numel() != cells(levels) * P:
        raise IHError("tmpl_desc must hold cells(levels) * P values")
    n = origins.shape[0]
    if dist is None:
        dist = torch.empty(n, dtype=torch.float32, device=ih.device)
    if best is None:
        best = torch.empty(1, dtype=torch.int32, device=ih.device)
    _dev(dist, "dist", torch.float32)
    _dev(best, "best", torch.int32)
    _check(lib().ih_match_candidates(_p(ih), P, H, W, _layout(layout), _p(tmpl_desc), win_h, win_w, levels,
                                     _p(origins), n, METRICS[metric], _p(dist), _p(best), _stream(ih)),
           "ih_match_candidates")
    return dist, best


def ih_profile_events(start: Optional[torch.cuda.Event], stop: Optional[torch.cuda.Event]):
    """Record `start`/`stop` around the final write-out kernel of later ih_build calls."""
    if start is None:
        _check(lib().ih_profile_events(None, None), "ih_profile_events")
    else:
        if not start.cuda_event or not stop.cuda_event:
            raise IHError("events must have been recorded once (torch creates them lazily)")
        _check(lib().ih_profile_events(ctypes.c_void_p(start.cuda_event), ctypes.c_void_p(stop.cuda_event)),
               "ih_profile_events")


class Batch:
    """Many frames of uneven size built (and searched) in one persistent launch.

    ``frames`` is a list of dicts with keys ``img`` (C x H x W uint8/uint16
    CUDA tensor), ``bins``, optional ``value_bits``, ``tile`` (TileCfg),
    and, for the candidate search, ``origins`` (n x 2 int32 tensor),
    ``win`` ((h, w)) and either ``tmpl_desc`` (21 x P int32 tensor) or
    ``tmpl_win`` ((r, c, h, w) in this frame), and optionally ``layout``
    (default: the batch's ``layout``).  Output tensors are allocated
    once; ``run()`` enqueues the batch on the current stream and may be
    captured in a CUDA (HIP) graph (phased mode).
    """

    def __init__(self, frames, metric: str = "chi2", layout: str = "bhw"):
        if not frames:
            raise IHError("empty batch")
        dt = frames[0]["img"].dtype
        if dt not in (torch.uint8, torch.uint16):
            raise IHError("img must be uint8 or uint16")
        self.dtype = IH_U8 if dt == torch.uint8 else IH_U16
        self.metric = METRICS[metric]
        n = len(frames)
        arr = (Frame * n)()
        self.ih, self.dist, self.best, self.tmpl, self._keep = [], [], [], [], []
        for i, fr in enumerate(frames):
            img = _dev(fr["img"], "img")
            if img.dim() == 2:
                img = img.unsqueeze(0)
            if img.dtype != dt:
                raise IHError("all frames of a batch share one dtype")
            C, H, W = img.shape
            bins = int(fr["bins"])
            bits = int(fr.get("value_bits", 8 if dt == torch.uint8 else 16))
            lay = fr.get("layout", layout)
            out = torch.empty(shape_of(C * bins, H, W, lay), dtype=torch.int32, device=img.device)
            a = arr[i]
            a.img, a.ih = img.data_ptr(), out.data_ptr()
            a.H, a.W, a.C, a.bins, a.value_bits = H, W, C, bins, bits
            a.layout = _layout(lay)
            if fr.get("tile") is not None:
                a.tile = fr["tile"]
            keep = [img, out]
            dist = best = tm = None
            if fr.get("origins") is not None:
                org = _dev(fr["origins"], "origins", torch.int32)
                nc = org.shape[0]
                dist = torch.empty(nc, dtype=torch.float32, device=img.device)
                best = torch.empty(1, dtype=torch.int32, device=img.device)
                a.origins, a.n_cand = org.data_ptr(), nc
                a.dist, a.best = dist.data_ptr(), best.data_ptr()
                a.win_h, a.win_w = (int(v) for v in fr["win"])
                if fr.get("tmpl_desc") is not None:
                    tm = _dev(fr["tmpl_desc"], "tmpl_desc", torch.int32)
                    a.tmpl_desc = tm.data_ptr()
                else:
                    tm = torch.empty((21, C * bins), dtype=torch.int32, device=img.device)
                    a.tmpl_out = tm.data_ptr()
                    for k, v in enumerate(fr["tmpl_win"]):
                        a.tmpl_win[k] = int(v)
                keep += [org, dist, best, tm]
            self.ih.append(out)
            self.dist.append(dist)
            self.best.append(best)
            self.tmpl.append(tm)
            self._keep.append(keep)
        self.frames = arr
        nbytes = lib().ih_batch_plan_bytes(n)
        self.plan_host = (ctypes.c_uint8 * nbytes)()
        ws = _SZ(0)
        _check(lib().ih_batch_plan(ctypes.byref(arr), n, self.dtype, self.metric, self.plan_host, nbytes,
                                   ctypes.byref(ws)), "ih_batch_plan")
        dev = frames[0]["img"].device
        self.plan_dev = torch.frombuffer(bytearray(self.plan_host), dtype=torch.uint8).to(dev)
        self.ws = torch.empty(max(1, ws.value), dtype=torch.uint8, device=dev)
        self.device = dev

    def run(self, mode: str = "phased"):
        """Enqueue the batch: ``"phased"`` (one launch per phase) or
        ``"cooperative"`` (one cooperative persistent launch)."""
        m = BATCH_MODES[mode]
        _check(lib().ih_build_batch(self.plan_host, _p(self.plan_dev), _p(self.ws), self.ws.numel(), m,
                                    _stream(self.ws)), "ih_build_batch")
