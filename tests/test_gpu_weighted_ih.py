"""GPU parity of ih_build_weighted (the magnitude-weighted orientation
histogram of Alg. 2 step 4) against the CPU oracle: bit-exact, both layouts,
every write-out form, with and without an edge mask."""
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


def case(seed, C, H, W, bits, mask_p=0.3):
    rng = np.random.default_rng(seed)
    dt = np.uint8 if bits <= 8 else np.uint16
    img = rng.integers(0, 1 << bits, size=(C, H, W)).astype(dt)
    wt = rng.integers(0, 256, size=(C, H, W)).astype(np.uint8)
    mask = np.where(rng.random((C, H, W)) < mask_p, 255, 0).astype(np.uint8)
    return img, wt, mask


SHAPES = [
    # C, H, W, bins, bits
    (1, 1, 1, 1, 8),
    (1, 1, 300, 4, 8),
    (1, 300, 1, 4, 8),
    (1, 97, 203, 8, 8),
    (2, 130, 301, 5, 16),
    (3, 64, 64, 256, 8),       # 768 planes: the unstaged planes-innermost write-out
    (1, 70, 1030, 16, 8),
    (7, 45, 77, 16, 8),
]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("C,H,W,bins,bits", SHAPES)
def test_weighted_bit_exact(C, H, W, bins, bits, layout):
    say("ih_build_weighted", layout, C, H, W, bins, bits)
    ih = ihlib()
    img, wt, mask = case(H * 7 + W + bins, C, H, W, bits)
    for m in (None, mask):
        out = ih.ih_build_weighted(gpu(img), bins, gpu(wt), gpu(m) if m is not None else None, bits,
                                   layout=layout)
        assert np.array_equal(bhw(out, layout), oracle.ih_weighted(img, bins, bits, wt, m)), m is None


def test_weighted_every_tile_shape():
    ih = ihlib()
    C, H, W, bins = 2, 150, 333, 16
    img, wt, mask = case(5, C, H, W, 8)
    ref = oracle.ih_weighted(img, bins, 8, wt, mask)
    t, tw_, tm = gpu(img), gpu(wt), gpu(mask)
    shapes = [("bhw", th, tw, pg) for th, tw, pg in itertools.product((1, 7, 32, 64, 128), (64, 128, 256),
                                                                      (1, 2, 4, 8, 16))]
    shapes += [("hwb", th, tw, 64) for th, tw in itertools.product((1, 7, 32, 64, 256), (16, 32, 64))]
    for layout, th, tw, pg in shapes:
        if th * tw > 32768:
            continue
        cfg = ih.TileCfg(th, tw, pg)
        say("tile", layout, cfg)
        if th * (tw + 4) * 2 > 64 * 1024 - 8 * max(th, tw):
            # the tile's bins and weights staged in LDS leave no room for a histogram
            with pytest.raises(ih.IHError, match="no LDS"):
                ih.ih_build_weighted(t, bins, tw_, tm, cfg=cfg, layout=layout)
            continue
        out = ih.ih_build_weighted(t, bins, tw_, tm, cfg=cfg, layout=layout)
        assert np.array_equal(bhw(out, layout), ref), (layout, cfg)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_weighted_unaligned_weight_rows(layout):
    """Weight and mask views that start one byte into their buffers, and an
    odd width, take the byte-wise load path."""
    ih = ihlib()
    for (H, W) in ((64, 256), (50, 203)):
        img, wt, mask = case(H + W, 1, H, W, 8)
        wbuf = torch.zeros(H * W + 1, dtype=torch.uint8, device=DEV)
        mbuf = torch.zeros(H * W + 1, dtype=torch.uint8, device=DEV)
        wbuf[1:] = gpu(wt.ravel())
        mbuf[1:] = gpu(mask.ravel())
        out = ih.ih_build_weighted(gpu(img), 16, wbuf[1:].view(1, H, W), mbuf[1:].view(1, H, W), layout=layout)
        assert np.array_equal(bhw(out, layout), oracle.ih_weighted(img, 16, 8, wt, mask)), (H, W)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_unit_weights_match_count_build(layout):
    ih = ihlib()
    img = synth.gray_u8(3, 211, 517)[None]
    t = gpu(img)
    ones = torch.ones_like(t)
    a = ih.ih_build_weighted(t, 32, ones, layout=layout)
    b = ih.ih_build(t, 32, layout=layout)
    assert torch.equal(a, b)


def test_weighted_errors():
    ih = ihlib()
    img = torch.zeros((1, 8, 8), dtype=torch.uint8, device=DEV)
    with pytest.raises(ih.IHError):
        ih.ih_build_weighted(img, 4, torch.zeros((1, 8, 7), dtype=torch.uint8, device=DEV))
    with pytest.raises(ih.IHError):
        ih.ih_build_weighted(img, 4, torch.zeros((1, 8, 8), dtype=torch.int32, device=DEV))
    # H * W * 255 above 2^31 - 1 is refused before any launch
    big = torch.zeros((1, 3000, 3000), dtype=torch.uint8, device=DEV)
    with pytest.raises(ih.IHError, match="overflow"):
        ih.ih_build_weighted(big, 1, big)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_phog_1920x1080_full(layout):
    """The 1920x1080 scene: orientation binned into 16 bins, magnitude as the
    weight, edge pixels only; the whole tensor against the oracle, then the
    three-level pyramid descriptors of windows taken from it."""
    ih = ihlib()
    go, gm, edge = synth.phog_inputs()
    say("phog 1920x1080x16", layout)
    out = ih.ih_build_weighted(gpu(go), 16, gpu(gm), gpu(edge), layout=layout)
    ref = oracle.ih_weighted(go, 16, 8, gm, edge)
    assert np.array_equal(bhw(out, layout), ref)
    wins = synth.rects_uniform(204, 1080, 1920, 2000, 16, 256)
    wins = np.stack([wins[:, 0], wins[:, 1], wins[:, 2] - wins[:, 0], wins[:, 3] - wins[:, 1]], 1).astype(np.int32)
    d = ih.ih_pyramid_desc(out, gpu(wins), 3, layout=layout).cpu().numpy()
    assert np.array_equal(d, oracle.pyramid_desc(ref, wins, 3))


def test_weighted_deterministic():
    ih = ihlib()
    go, gm, edge = synth.phog_inputs(scale=0.25)
    t, w, m = gpu(go), gpu(gm), gpu(edge)
    for layout in LAYOUTS:
        first = ih.ih_build_weighted(t, 16, w, m, layout=layout)
        for i in range(10):
            assert torch.equal(first, ih.ih_build_weighted(t, 16, w, m, layout=layout)), (layout, i)
