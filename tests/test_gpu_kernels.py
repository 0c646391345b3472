"""GPU parity of the further spatial kernels: second-moment integral
histograms (bit-exact modulo 2^32), the quadratic kernel in O(1) (bit-exact
against the oracle's integer route, within 1e-5 of its FP64 brute force) and
the wedding cake of Eq. 3.2 (within FP32 rounding of the oracle's FP64)."""
import itertools

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LAYOUTS = ["bhw", "hwb"]


def ihlib():
    import paper_1711_01656_amd as ih
    return ih


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(*a):
    print(*a, flush=True)


def bhw(t, layout):
    a = t.cpu().numpy()
    return a if layout == "bhw" else np.ascontiguousarray(a.transpose(2, 0, 1))


def mod32(a):
    return np.asarray(a).astype(np.int64) & 0xFFFFFFFF


def rand_img(seed, C, H, W, bits):
    rng = np.random.default_rng(seed)
    dt = np.uint8 if bits <= 8 else np.uint16
    return rng.integers(0, 1 << bits, size=(C, H, W)).astype(dt)


def rects_of(seed, H, W, n, lo=1, hi=64):
    rng = np.random.default_rng(seed)
    h = rng.integers(lo, min(hi, H) + 1, n)
    w = rng.integers(lo, min(hi, W) + 1, n)
    r0 = (rng.random(n) * (H - h + 1)).astype(np.int64)
    c0 = (rng.random(n) * (W - w + 1)).astype(np.int64)
    return np.stack([r0, c0, r0 + h, c0 + w], 1).astype(np.int32)


SHAPES = [(1, 1, 1, 1, 8), (1, 97, 203, 8, 8), (2, 130, 301, 5, 16), (3, 64, 64, 256, 8), (7, 45, 77, 16, 8)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("C,H,W,bins,bits", SHAPES)
def test_moments2_exact_mod_2_32(C, H, W, bins, bits, layout):
    say("moments2", layout, C, H, W, bins, bits)
    ih = ihlib()
    img = rand_img(H + W, C, H, W, bits)
    mxx, myy = ih.ih_build_moments2(gpu(img), bins, bits, layout=layout)
    oxx, oyy = oracle.moments2(img, bins, bits)
    assert np.array_equal(mod32(bhw(mxx, layout)), mod32(oxx))
    assert np.array_equal(mod32(bhw(myy, layout)), mod32(oyy))


def test_moments2_every_tile_shape():
    ih = ihlib()
    C, H, W, bins = 2, 150, 333, 16
    img = rand_img(5, C, H, W, 8)
    oxx, oyy = oracle.moments2(img, bins, 8)
    t = gpu(img)
    shapes = [("bhw", th, tw, pg) for th, tw, pg in itertools.product((1, 7, 32, 128), (64, 128, 256), (1, 4, 16))]
    shapes += [("hwb", th, tw, 64) for th, tw in itertools.product((1, 7, 32, 256), (16, 32, 64))]
    for layout, th, tw, pg in shapes:
        if th * tw > 32768:
            continue
        cfg = ih.TileCfg(th, tw, pg)
        say("tile", layout, cfg)
        mxx, myy = ih.ih_build_moments2(t, bins, cfg=cfg, layout=layout)
        assert np.array_equal(mod32(bhw(mxx, layout)), mod32(oxx)), cfg
        assert np.array_equal(mod32(bhw(myy, layout)), mod32(oyy)), cfg


def five(img, bins, bits, layout):
    ih = ihlib()
    t = gpu(img)
    c, mx, my = ih.ih_build(t, bins, bits, moments=True, layout=layout)
    mxx, myy = ih.ih_build_moments2(t, bins, bits, layout=layout)
    return c, mx, my, mxx, myy


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("l1", [False, True])
def test_quadratic_query_matches_oracle(layout, l1):
    ih = ihlib()
    C, H, W, bins = 2, 140, 260, 8
    img = rand_img(7, C, H, W, 8)
    rects = rects_of(8, H, W, 3000, 1, 140)
    extra = np.array([[0, 0, H, W], [5, 5, 5, 9], [3, 4, 4, 5], [0, 0, 0, 0], [H - 1, W - 1, H, W]], np.int32)
    rects = np.concatenate([rects, extra])
    c, mx, my, mxx, myy = five(img, bins, 8, layout)
    out = ih.ih_query_quadratic(c, mx, my, mxx, myy, C, gpu(rects), l1, layout=layout).cpu().numpy()
    ih_o = oracle.ih(img, bins, 8)
    omx, omy = oracle.moments(img, bins, 8)
    oxx, oyy = oracle.moments2(img, bins, 8)
    _, ref = oracle.quadratic_swih(ih_o, omx, omy, oxx, oyy, C, rects, l1)
    assert np.array_equal(out, ref)
    bf = oracle.kernel_bruteforce(img, bins, 8, rects, "quadratic", l1norm=l1)
    nz = np.abs(bf) > 0
    assert np.all(np.abs(out[nz] - bf[nz]) <= 1e-5 * np.abs(bf[nz]))
    assert np.all(out[~nz] == 0)


def test_quadratic_query_invalid_and_large_windows():
    ih = ihlib()
    H, W = 3000, 40
    img = rand_img(9, 1, H, W, 8)
    c, mx, my, mxx, myy = five(img, 4, 8, "bhw")
    rects = np.array([[0, 0, 2400, 1], [0, 0, 2300, 1], [-1, 0, 3, 3], [0, 0, 3001, 3], [2, 3, 1, 5]], np.int32)
    out = ih.ih_query_quadratic(c, mx, my, mxx, myy, 1, gpu(rects)).cpu().numpy()
    # a 2400 x 1 window reaches w (h-1) h (2h-1) / 6 >= 2^32: NaN; 2300 x 1 is exact
    assert np.isnan(out[0]).all() and not np.isnan(out[1]).any()
    assert np.isnan(out[2:]).all()
    num = oracle.quadratic_numerator(img, 4, 8, rects[1:2])
    den = 2.0 * 2300 ** 2
    assert np.array_equal(out[1], (num[0] / den).astype(np.float32))


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("kernel,sigma", [("manhattan", 0.5), ("quadratic", 0.5), ("gaussian", 0.5),
                                          ("gaussian", 0.25)])
def test_wedding_matches_oracle(layout, kernel, sigma):
    ih = ihlib()
    C, H, W, bins = 3, 120, 200, 16
    img = rand_img(11, C, H, W, 8)
    rects = np.concatenate([rects_of(12, H, W, 1500, 1, 120),
                            np.array([[0, 0, 0, 5], [-1, 0, 4, 4], [0, 0, H, W]], np.int32)])
    t = ih.ih_build(gpu(img), bins, layout=layout)
    ih_o = oracle.ih(img, bins, 8)
    for L in (1, 2, 3, 5, 8, 16):
        out = ih.ih_query_wedding(t, C, gpu(rects), L, kernel, sigma, layout=layout).cpu().numpy()
        ref = oracle.wedding(ih_o, rects, L, kernel, sigma)
        fin = np.isfinite(ref)
        assert np.array_equal(np.isnan(out), ~fin)
        np.testing.assert_allclose(out[fin], ref[fin], rtol=1e-6, atol=1e-6, err_msg="L=%d" % L)


def test_wedding_errors():
    ih = ihlib()
    t = torch.zeros((4, 8, 8), dtype=torch.int32, device=DEV)
    r = gpu(np.array([[0, 0, 4, 4]], np.int32))
    for bad in (dict(layers=0), dict(layers=17), dict(kernel="gaussian", sigma=0.0)):
        args = dict(layers=3, kernel="manhattan", sigma=0.5)
        args.update(bad)
        with pytest.raises(ih.IHError):
            ih.ih_query_wedding(t, 1, r, args["layers"], args["kernel"], args["sigma"])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_config2_frame_sampled(layout):
    """The 1920x1080x7-channel frame with 16 bins: quadratic-kernel histograms
    of 2,000 of its windows against the oracle's brute-force integer
    numerators, and wedding cakes against the oracle's FP64 from its count IH
    planes."""
    ih = ihlib()
    w = synth.config2(n_windows=2000)
    say("config2 quadratic + wedding", layout)
    c, mx, my, mxx, myy = five(w.img, w.bins, w.bits, layout)
    rects = w.windows
    out = ih.ih_query_quadratic(c, mx, my, mxx, myy, w.C, gpu(rects), layout=layout).cpu().numpy()
    num = oracle.quadratic_numerator(w.img, w.bins, w.bits, rects)
    h = (rects[:, 2] - rects[:, 0]).astype(np.float64)
    ww = (rects[:, 3] - rects[:, 1]).astype(np.float64)
    ref = (num / (2 * h * h * ww * ww)[:, None]).astype(np.float32)
    assert np.array_equal(out, ref)
    wed = ih.ih_query_wedding(c, w.C, gpu(rects), 3, "gaussian", 0.5, layout=layout).cpu().numpy()
    bf = oracle.wedding_direct(w.img, w.bins, w.bits, rects[:300], 3, "gaussian", 0.5)
    np.testing.assert_allclose(wed[:300], bf, rtol=1e-6, atol=1e-6)
