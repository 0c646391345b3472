"""CPU oracle for the integral-histogram path (test infrastructure only).

A plain, slow, obviously-correct implementation of what the GPU path computes,
written from the thesis's definitions (Poostchi 2017, arXiv:1711.01656): the
C file ``ih_oracle.c`` holds the arithmetic, this module only marshals numpy
arrays into it (plus the NumPy FP64 CNN oracle in ``cnn.py``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product library never imports it, and this
package imports nothing from the product: the two share no code.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ih_oracle.c")
_LIB = os.path.join(_HERE, "libih_oracle.so")
_lock = threading.Lock()
_lib = None

U8, U16 = 0, 1
CHI2, L1, PMK = 0, 1, 2
METRICS = {"chi2": CHI2, "l1": L1, "pmk": PMK}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP) into ``oracle/libih_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            I = ctypes.c_int
            I64 = ctypes.c_int64
            D = ctypes.c_double
            sig = {
                "or_check_values": [P, I, I, I, I, I],
                "or_plane_index": [P, I, I, I, I, I, I, P],
                "or_ih_plane": [P, I, I, I, I, I, I, I, P],
                "or_ih": [P, I, I, I, I, I, I, P],
                "or_ih_bruteforce": [P, I, I, I, I, I, I, P],
                "or_moments_plane": [P, I, I, I, I, I, I, I, P, P],
                "or_moments": [P, I, I, I, I, I, I, P, P],
                "or_query_rect": [P, I, I, I, P, I64, P],
                "or_query_rect_direct": [P, I, I, I, I, I, I, P, I64, P],
                "or_weighted_bruteforce": [P, I, I, I, I, I, I, P, I64, I, P],
                "or_weighted_numerator": [P, I, I, I, I, I, I, P, I64, P],
                "or_weighted_swih": [P, P, P, I, I, I, I, P, I64, I, P, P],
                "or_pyramid_desc": [P, I, I, I, P, I64, I, P],
                "or_pyramid_desc_direct": [P, I, I, I, I, I, I, P, I64, I, P],
                "or_pyramid_distance": [P, P, I, I, I],
                "or_match_direct": [P, I, I, I, I, I, I, P, I, I, I, P, I64, I, P, P],
                "or_level_weight": [I, I],
                "or_num_threads": [],
                "or_ih_weighted": [P, I, P, P, I, I, I, I, I, P],
                "or_color_likelihood": [P, I, I, P, P, P, P],
                "or_moment_images": [P, I, I, P, P, P],
                "or_camshift": [P, I, I, P, I64, I, I, D, I, P, P],
                "or_kernel_bruteforce": [P, I, I, I, I, I, I, P, I64, I, D, I, P],
                "or_moments2": [P, I, I, I, I, I, I, P, P],
                "or_quadratic_numerator": [P, I, I, I, I, I, I, P, I64, P],
                "or_quadratic_swih": [P, P, P, P, P, I, I, I, I, P, I64, I, P, P],
                "or_ring_weights": [I, I, I, I, D, P],
                "or_wedding": [P, I, I, I, P, I64, I, I, D, P],
                "or_wedding_direct": [P, I, I, I, I, I, I, P, I64, I, I, D, P],
                "or_jih": [P, I, I, I, I, I, I, I, P],
                "or_st_median": [P, I, I, I, I, I, I, I, I, I, P],
                "or_ih_weighted_bruteforce": [P, I, P, P, I, I, I, I, I, P],
                "or_set_threads": [I],
            }
            for name, args in sig.items():
                f = getattr(lib, name)
                f.argtypes = args
                f.restype = ctypes.c_int
            lib.or_pyramid_distance.restype = ctypes.c_double
            lib.or_level_weight.restype = ctypes.c_double
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError("oracle %s failed with code %d" % (what, rc))


def _img(img: np.ndarray):
    """Return (contiguous C x H x W array, dtype code, C, H, W)."""
    a = np.ascontiguousarray(img)
    if a.ndim == 2:
        a = a[None]
    if a.dtype == np.uint8:
        dt = U8
    elif a.dtype == np.uint16:
        dt = U16
    else:
        raise TypeError("image must be uint8 or uint16, got %s" % a.dtype)
    C, H, W = a.shape
    return a, dt, C, H, W


def num_threads() -> int:
    return _load().or_num_threads()


def set_threads(n: int) -> int:
    """Threads for later oracle calls (n < 1 restores the default); returns the count."""
    return _load().or_set_threads(int(n))


def cells(levels: int) -> int:
    return sum(4 ** l for l in range(levels))


def check_values(img, bits):
    a, dt, C, H, W = _img(img)
    return _load().or_check_values(_ptr(a), dt, H, W, C, bits) == 0


def plane_index(img, bins, bits):
    a, dt, C, H, W = _img(img)
    out = np.empty((C, H, W), np.int32)
    _check(_load().or_plane_index(_ptr(a), dt, H, W, C, bins, bits, _ptr(out)), "plane_index")
    return out


def ih(img, bins, bits):
    """Integral histogram P x H x W int32 by the Alg. 5 recurrence."""
    a, dt, C, H, W = _img(img)
    out = np.empty((C * bins, H, W), np.int32)
    _check(_load().or_ih(_ptr(a), dt, H, W, C, bins, bits, _ptr(out)), "ih")
    return out


def _u8(a, shape, name):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    if a.shape != shape:
        raise ValueError("%s must have shape %s" % (name, shape))
    return a


def ih_weighted(img, bins, bits, weight, mask=None, brute=False):
    """Weighted integral histogram (Alg. 2 step 4): plane k accumulates the
    pixel's weight where its bin is k and its mask is set.  P x H x W int32."""
    a, dt, C, H, W = _img(img)
    w = _u8(weight, (C, H, W), "weight")
    m = None if mask is None else _u8(mask, (C, H, W), "mask")
    out = np.empty((C * bins, H, W), np.int32)
    fn = _load().or_ih_weighted_bruteforce if brute else _load().or_ih_weighted
    _check(fn(_ptr(a), dt, _ptr(w), _ptr(m) if m is not None else None, H, W, C, bins, bits, _ptr(out)),
           "ih_weighted")
    return out


def _frames(frames):
    """F x C x H x W (or F x H x W) uint8/uint16 stack -> (array, dtype code, F, C, H, W)."""
    a = np.ascontiguousarray(frames)
    if a.ndim == 3:
        a = a[:, None]
    if a.ndim != 4:
        raise ValueError("frames must be F x C x H x W")
    if a.dtype == np.uint8:
        dt = U8
    elif a.dtype == np.uint16:
        dt = U16
    else:
        raise TypeError("frames must be uint8 or uint16, got %s" % a.dtype)
    F, C, H, W = a.shape
    return a, dt, F, C, H, W


def jih(frames, bins, bits):
    """Joint integral histogram of a temporal window of frames (Alg. 4): the
    integral histogram of all the window's pixels.  P x H x W int32."""
    a, dt, F, C, H, W = _frames(frames)
    out = np.empty((C * bins, H, W), np.int32)
    _check(_load().or_jih(_ptr(a), dt, F, H, W, C, bins, bits, _ptr(out)), "jih")
    return out


def st_median(frames, bins, bits, win_h, win_w):
    """Spatio-temporal median (Alg. 4, Sec. 4.1.1) by its definition: the lower
    median of the binned samples of each pixel's clipped win_h x win_w window
    over all frames.  C x H x W int32 bin indices."""
    a, dt, F, C, H, W = _frames(frames)
    out = np.empty((C, H, W), np.int32)
    _check(_load().or_st_median(_ptr(a), dt, F, H, W, C, bins, bits, win_h, win_w, _ptr(out)), "st_median")
    return out


def ih_plane(img, bins, bits, p):
    a, dt, C, H, W = _img(img)
    out = np.empty((H, W), np.int32)
    _check(_load().or_ih_plane(_ptr(a), dt, H, W, C, bins, bits, p, _ptr(out)), "ih_plane")
    return out


def ih_bruteforce(img, bins, bits):
    """Eq. 2.15 as the explicit double sum (tiny images only)."""
    a, dt, C, H, W = _img(img)
    out = np.empty((C * bins, H, W), np.int32)
    _check(_load().or_ih_bruteforce(_ptr(a), dt, H, W, C, bins, bits, _ptr(out)), "ih_bruteforce")
    return out


def moments(img, bins, bits):
    """Coordinate-moment integral histograms (Mx, My), each P x H x W int64."""
    a, dt, C, H, W = _img(img)
    mx = np.empty((C * bins, H, W), np.int64)
    my = np.empty((C * bins, H, W), np.int64)
    _check(_load().or_moments(_ptr(a), dt, H, W, C, bins, bits, _ptr(mx), _ptr(my)), "moments")
    return mx, my


def moments_plane(img, bins, bits, p):
    a, dt, C, H, W = _img(img)
    mx = np.empty((H, W), np.int64)
    my = np.empty((H, W), np.int64)
    _check(_load().or_moments_plane(_ptr(a), dt, H, W, C, bins, bits, p, _ptr(mx), _ptr(my)),
           "moments_plane")
    return mx, my


def _rects(rects):
    r = np.ascontiguousarray(np.asarray(rects, dtype=np.int32).reshape(-1, 4))
    return r, r.shape[0]


def query_rect(ihist, rects):
    """Eq. 2.16 on a P x H x W integral histogram; rects are {r0, c0, r1, c1}."""
    t = np.ascontiguousarray(ihist, dtype=np.int32)
    P, H, W = t.shape
    r, n = _rects(rects)
    out = np.empty((n, P), np.int32)
    _check(_load().or_query_rect(_ptr(t), P, H, W, _ptr(r), n, _ptr(out)), "query_rect")
    return out


def query_rect_direct(img, bins, bits, rects):
    a, dt, C, H, W = _img(img)
    r, n = _rects(rects)
    out = np.empty((n, C * bins), np.int32)
    _check(_load().or_query_rect_direct(_ptr(a), dt, H, W, C, bins, bits, _ptr(r), n, _ptr(out)),
           "query_rect_direct")
    return out


def weighted_bruteforce(img, bins, bits, rects, l1norm=False):
    """Eq. 3.1 with the Manhattan kernel, FP64 brute force; n x P float64."""
    a, dt, C, H, W = _img(img)
    r, n = _rects(rects)
    out = np.empty((n, C * bins), np.float64)
    _check(_load().or_weighted_bruteforce(_ptr(a), dt, H, W, C, bins, bits, _ptr(r), n,
                                          int(bool(l1norm)), _ptr(out)), "weighted_bruteforce")
    return out


def weighted_numerator(img, bins, bits, rects):
    a, dt, C, H, W = _img(img)
    r, n = _rects(rects)
    out = np.empty((n, C * bins), np.int64)
    _check(_load().or_weighted_numerator(_ptr(a), dt, H, W, C, bins, bits, _ptr(r), n, _ptr(out)),
           "weighted_numerator")
    return out


def weighted_swih(ihist, mx, my, C, rects, l1norm=False):
    """SWIH quadrant decomposition (Sec. 3.1.3): (int64 numerators, float32 values)."""
    t = np.ascontiguousarray(ihist, dtype=np.int32)
    mx = np.ascontiguousarray(mx, dtype=np.int64)
    my = np.ascontiguousarray(my, dtype=np.int64)
    P, H, W = t.shape
    r, n = _rects(rects)
    num = np.empty((n, P), np.int64)
    out = np.empty((n, P), np.float32)
    _check(_load().or_weighted_swih(_ptr(t), _ptr(mx), _ptr(my), P, H, W, C, _ptr(r), n,
                                    int(bool(l1norm)), _ptr(num), _ptr(out)), "weighted_swih")
    return num, out


KERNELS = {"manhattan": 0, "quadratic": 1, "gaussian": 2}


def kernel_bruteforce(img, bins, bits, rects, kernel="manhattan", sigma=0.5, l1norm=False):
    """Eq. 3.1 by brute force in FP64 with the Manhattan, quadratic or Gaussian
    kernel (normalised window coordinates); n x P float64."""
    a, dt, C, H, W = _img(img)
    r, n = _rects(rects)
    out = np.empty((n, C * bins), np.float64)
    _check(_load().or_kernel_bruteforce(_ptr(a), dt, H, W, C, bins, bits, _ptr(r), n, KERNELS[kernel],
                                        float(sigma), int(bool(l1norm)), _ptr(out)), "kernel_bruteforce")
    return out


def moments2(img, bins, bits):
    """Second coordinate-moment integral histograms (Mxx, Myy), P x H x W int64."""
    a, dt, C, H, W = _img(img)
    mxx = np.empty((C * bins, H, W), np.int64)
    myy = np.empty((C * bins, H, W), np.int64)
    _check(_load().or_moments2(_ptr(a), dt, H, W, C, bins, bits, _ptr(mxx), _ptr(myy)), "moments2")
    return mxx, myy


def quadratic_numerator(img, bins, bits, rects):
    a, dt, C, H, W = _img(img)
    r, n = _rects(rects)
    out = np.empty((n, C * bins), np.int64)
    _check(_load().or_quadratic_numerator(_ptr(a), dt, H, W, C, bins, bits, _ptr(r), n, _ptr(out)),
           "quadratic_numerator")
    return out


def quadratic_swih(ihist, mx, my, mxx, myy, C, rects, l1norm=False):
    """The quadratic kernel from five integral histograms: (int64 numerators, float32 values)."""
    t = np.ascontiguousarray(ihist, dtype=np.int32)
    arrs = [np.ascontiguousarray(m, dtype=np.int64) for m in (mx, my, mxx, myy)]
    P, H, W = t.shape
    r, n = _rects(rects)
    num = np.empty((n, P), np.int64)
    out = np.empty((n, P), np.float32)
    _check(_load().or_quadratic_swih(_ptr(t), *[_ptr(m) for m in arrs], P, H, W, C, _ptr(r), n,
                                     int(bool(l1norm)), _ptr(num), _ptr(out)), "quadratic_swih")
    return num, out


def ring_weights(h, w, layers, kernel="manhattan", sigma=0.5):
    """The wedding cake's ring weights (Eq. 3.2) for an h x w window."""
    out = np.empty(layers, np.float64)
    _check(_load().or_ring_weights(h, w, layers, KERNELS[kernel], float(sigma), _ptr(out)), "ring_weights")
    return out


def wedding(ihist, rects, layers, kernel="manhattan", sigma=0.5):
    """Wedding-cake approximation (Eq. 3.2) from the count IH; n x P float64."""
    t = np.ascontiguousarray(ihist, dtype=np.int32)
    P, H, W = t.shape
    r, n = _rects(rects)
    out = np.empty((n, P), np.float64)
    _check(_load().or_wedding(_ptr(t), P, H, W, _ptr(r), n, layers, KERNELS[kernel], float(sigma), _ptr(out)),
           "wedding")
    return out


def wedding_direct(img, bins, bits, rects, layers, kernel="manhattan", sigma=0.5):
    """The wedding-cake approximation by direct per-pixel ring counting; n x P float64."""
    a, dt, C, H, W = _img(img)
    r, n = _rects(rects)
    out = np.empty((n, C * bins), np.float64)
    _check(_load().or_wedding_direct(_ptr(a), dt, H, W, C, bins, bits, _ptr(r), n, layers, KERNELS[kernel],
                                     float(sigma), _ptr(out)), "wedding_direct")
    return out


def color_likelihood(rgb, fg, bg):
    """FG/BG colour likelihood (Eq. 2.18-2.21) of a 3 x H x W uint8 image:
    (q, L) with q the uint8 code round(255 L) taken in integers and L in FP64."""
    a = np.ascontiguousarray(rgb, dtype=np.uint8)
    if a.ndim != 3 or a.shape[0] != 3:
        raise ValueError("rgb must be 3 x H x W")
    _, H, W = a.shape
    f = np.ascontiguousarray(fg, dtype=np.int32).reshape(4)
    b = np.ascontiguousarray(bg, dtype=np.int32).reshape(4)
    q = np.empty((H, W), np.uint8)
    L = np.empty((H, W), np.float64)
    _check(_load().or_color_likelihood(_ptr(a), H, W, _ptr(f), _ptr(b), _ptr(q), _ptr(L)), "color_likelihood")
    return q, L


def moment_images(q):
    """Integral images of q, row*q and column*q (int64 H x W each)."""
    a = np.ascontiguousarray(q, dtype=np.uint8)
    H, W = a.shape
    S, Sx, Sy = (np.empty((H, W), np.int64) for _ in range(3))
    _check(_load().or_moment_images(_ptr(a), H, W, _ptr(S), _ptr(Sx), _ptr(Sy)), "moment_images")
    return S, Sx, Sy


def camshift(q, starts, win_h, win_w, delta=0.5, max_iter=20):
    """CAMSHIFT (Alg. 1) with direct window sums: (n x 2 centres, n iterations)."""
    a = np.ascontiguousarray(q, dtype=np.uint8)
    H, W = a.shape
    st = np.ascontiguousarray(starts, dtype=np.float64).reshape(-1, 2)
    n = st.shape[0]
    cen = np.empty((n, 2), np.float64)
    it = np.empty(n, np.int32)
    _check(_load().or_camshift(_ptr(a), H, W, _ptr(st), n, win_h, win_w, float(delta), max_iter, _ptr(cen),
                               _ptr(it)), "camshift")
    return cen, it


def _wins(wins):
    w = np.ascontiguousarray(np.asarray(wins, dtype=np.int32).reshape(-1, 4))
    return w, w.shape[0]


def pyramid_desc(ihist, wins, levels):
    """Pyramid descriptors from an IH; wins are {r, c, h, w}; n x cells x P."""
    t = np.ascontiguousarray(ihist, dtype=np.int32)
    P, H, W = t.shape
    w, n = _wins(wins)
    out = np.empty((n, cells(levels), P), np.int32)
    _check(_load().or_pyramid_desc(_ptr(t), P, H, W, _ptr(w), n, levels, _ptr(out)), "pyramid_desc")
    return out


def pyramid_desc_direct(img, bins, bits, wins, levels):
    a, dt, C, H, W = _img(img)
    w, n = _wins(wins)
    out = np.empty((n, cells(levels), C * bins), np.int32)
    _check(_load().or_pyramid_desc_direct(_ptr(a), dt, H, W, C, bins, bits, _ptr(w), n, levels,
                                          _ptr(out)), "pyramid_desc_direct")
    return out


def level_weight(levels, l):
    return _load().or_level_weight(levels, l)


def pyramid_distance(a, b, levels, metric="chi2"):
    a = np.ascontiguousarray(a, dtype=np.int32)
    b = np.ascontiguousarray(b, dtype=np.int32)
    P = a.size // cells(levels)
    return _load().or_pyramid_distance(_ptr(a), _ptr(b), P, levels, METRICS[metric])


def match_direct(img, bins, bits, tmpl, win_h, win_w, levels, origins, metric="chi2"):
    """Exhaustive candidate search: (n distances float64, best index)."""
    a, dt, C, H, W = _img(img)
    t = np.ascontiguousarray(tmpl, dtype=np.int32)
    o = np.ascontiguousarray(np.asarray(origins, dtype=np.int32).reshape(-1, 2))
    n = o.shape[0]
    dist = np.empty(n, np.float64)
    best = np.zeros(1, np.int32)
    _check(_load().or_match_direct(_ptr(a), dt, H, W, C, bins, bits, _ptr(t), win_h, win_w, levels,
                                   _ptr(o), n, METRICS[metric], _ptr(dist), _ptr(best)),
           "match_direct")
    return dist, int(best[0])
