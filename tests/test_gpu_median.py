"""GPU parity of the spatio-temporal median path (Alg. 4): the in-place joint
integral histogram update (bit-exact against the oracle's joint IH of the
window after every push, in the cumulative-plane form the GPU stores), the
local median from a joint IH (bit-exact against the oracle's median of the
samples) and the streaming model end to end, both layouts."""
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


def to_layout(a, layout):
    return a if layout == "bhw" else np.ascontiguousarray(a.transpose(1, 2, 0))


def cum(J, C, bins):
    """Joint IH with cumulative planes (plane k counts bins <= k), as the GPU
    stores it, from the oracle's plain joint IH."""
    P, H, W = J.shape
    return J.reshape(C, bins, H, W).cumsum(axis=1, dtype=np.int64).reshape(P, H, W).astype(np.int32)


def video(seed, F, C, H, W, bits):
    rng = np.random.default_rng(seed)
    dt = np.uint8 if bits <= 8 else np.uint16
    v = rng.integers(0, 1 << bits, size=(F, C, H, W)).astype(dt)
    # repeat some pixels across frames so that head and tail share bins
    keep = rng.random((F, C, H, W)) < 0.4
    v[1:][keep[1:]] = v[:-1][keep[1:]]
    return v


UPDATE_SHAPES = [
    # C, H, W, bins, bits
    (1, 1, 1, 4, 8),
    (1, 97, 203, 16, 8),
    (2, 130, 301, 5, 10),
    (1, 64, 64, 256, 8),
    (3, 45, 77, 16, 8),
    (1, 33, 1030, 8, 16),
    (2, 50, 90, 100, 8),      # two channels, each with two 64-bin chunks in the tile pass
    (1, 21, 300, 256, 16),    # four chunks from 16-bit values
]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("C,H,W,bins,bits", UPDATE_SHAPES)
def test_jih_update_tracks_window(C, H, W, bins, bits, layout):
    say("jih update", layout, C, H, W, bins, bits)
    ih = ihlib()
    T1 = 4                                      # window of 4 frames
    v = video(H + W + bins, 9, C, H, W, bits)
    J = torch.zeros(ih.shape_of(C * bins, H, W, layout), dtype=torch.int32, device=DEV)
    for f in range(v.shape[0]):
        tail = gpu(v[f - T1]) if f >= T1 else None
        ih.ih_jih_update(gpu(v[f]), tail, bins, J, bits, layout=layout)
        lo = max(0, f - T1 + 1)
        assert np.array_equal(bhw(J, layout), cum(oracle.jih(v[lo:f + 1], bins, bits), C, bins)), f


def test_jih_update_every_tile_shape():
    ih = ihlib()
    C, H, W, bins = 2, 150, 333, 16
    v = video(11, 3, C, H, W, 8)
    base = cum(oracle.jih(v[0:2], bins, 8), C, bins)
    ref = cum(oracle.jih(v[1:3], bins, 8), C, bins)
    shapes = [("bhw", th, tw, pg) for th, tw, pg in itertools.product((1, 7, 32, 64, 128), (64, 128, 256),
                                                                      (1, 2, 4, 8, 16))]
    shapes += [("hwb", th, tw, 64) for th, tw in itertools.product((1, 7, 32, 64, 256), (16, 32, 64))]
    h, t = gpu(v[2]), gpu(v[0])
    for layout, th, tw, pg in shapes:
        if th * tw > 32768:
            continue
        cfg = ih.TileCfg(th, tw, pg)
        say("tile", layout, cfg)
        J = gpu(to_layout(base, layout))
        if th * (tw + 4) * 2 > 64 * 1024 - 4 * max(th, tw) * 2:
            with pytest.raises(ih.IHError, match="no LDS"):
                ih.ih_jih_update(h, t, bins, J, cfg=cfg, layout=layout)
            continue
        ih.ih_jih_update(h, t, bins, J, cfg=cfg, layout=layout)
        assert np.array_equal(bhw(J, layout), ref), (layout, cfg)


def test_jih_update_many_chunks_every_tile_shape():
    """The update's tile pass splits the bins into 64-bin chunks, each a
    block that starts from the counts of the lower bins; 150 bins over two
    channels make three uneven chunks per channel."""
    ih = ihlib()
    C, H, W, bins = 2, 70, 203, 150
    v = video(13, 3, C, H, W, 8)
    base = cum(oracle.jih(v[0:2], bins, 8), C, bins)
    ref = cum(oracle.jih(v[1:3], bins, 8), C, bins)
    h, t = gpu(v[2]), gpu(v[0])
    for layout, th, tw, pg in [("bhw", 1, 64, 1), ("bhw", 16, 128, 8), ("bhw", 64, 256, 4), ("bhw", 7, 128, 16),
                               ("hwb", 16, 32, 64), ("hwb", 64, 16, 64), ("hwb", 1, 32, 64)]:
        cfg = ih.TileCfg(th, tw, pg)
        say("chunks", layout, cfg)
        J = gpu(to_layout(base, layout))
        ih.ih_jih_update(h, t, bins, J, cfg=cfg, layout=layout)
        assert np.array_equal(bhw(J, layout), ref), (layout, cfg)


def test_jih_update_same_frame_is_identity_and_unaligned_output():
    ih = ihlib()
    v = video(12, 2, 1, 40, 257, 8)
    base = cum(oracle.jih(v, 8, 8), 1, 8)
    flat = torch.empty(8 * 40 * 257 + 1, dtype=torch.int32, device=DEV)
    J = flat[1:].view(8, 40, 257)                # 4-byte aligned, not 16
    J.copy_(gpu(base))
    f = gpu(v[1])
    ih.ih_jih_update(f, f, 8, J, cfg=ih.TileCfg(16, 256, 4))
    assert np.array_equal(J.cpu().numpy(), base)
    ih.ih_jih_update(gpu(v[0]), f, 8, J, cfg=ih.TileCfg(16, 256, 4))
    assert np.array_equal(J.cpu().numpy(), cum(oracle.jih(v[[0, 0]], 8, 8), 1, 8))


MEDIAN_CASES = [
    # C, H, W, bins, frames, win_h, win_w
    (1, 1, 1, 4, 1, 1, 1),
    (1, 9, 13, 16, 1, 1, 1),
    (1, 37, 53, 16, 3, 3, 3),
    (2, 40, 70, 32, 5, 5, 3),
    (1, 31, 29, 256, 17, 3, 3),
    (1, 20, 30, 100, 4, 2, 6),       # even windows, 100 bins (two 64-bin chunks)
    (1, 6, 7, 8, 2, 15, 15),         # window larger than the image
    (1, 25, 25, 1, 3, 3, 3),         # one bin: the median is always 0
]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("C,H,W,bins,frames,wh,ww", MEDIAN_CASES)
def test_local_median_matches_oracle(C, H, W, bins, frames, wh, ww, layout):
    say("median", layout, C, H, W, bins, frames, wh, ww)
    ih = ihlib()
    v = video(H * W + frames, frames, C, H, W, 8)
    J = gpu(to_layout(cum(oracle.jih(v, bins, 8), C, bins), layout))
    m = ih.ih_local_median(J, C, bins, frames, wh, ww, layout=layout)
    assert np.array_equal(m.cpu().numpy(), oracle.st_median(v, bins, 8, wh, ww))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_streaming_model_matches_oracle(layout):
    from paper_1711_01656_amd.median import SpatioTemporalMedian
    F, T, H, W, bins = 14, 6, 70, 90, 64
    v = synth.surveillance_video(21, F, H, W, n_movers=3)
    model = SpatioTemporalMedian(1, H, W, bins, T, 3, 3, layout=layout)
    seen = 0
    for f in range(F):
        r = model.push(gpu(v[f]))
        if f < T:
            assert r is None
            continue
        idx, med = r
        assert idx == f - T // 2
        ref = oracle.st_median(v[f - T:f + 1, None], bins, 8, 3, 3)
        assert np.array_equal(med.cpu().numpy(), ref), f
        seen += 1
    assert seen == F - T


@pytest.mark.parametrize("layout", LAYOUTS)
def test_surveillance_768x576_256bins(layout):
    """The benchmark workload: 768x576 grey video, 256 bins, a 17-frame window
    and a 3x3 spatial window; two medians compared in full with the oracle."""
    from paper_1711_01656_amd.median import SpatioTemporalMedian
    F, T = 19, 16
    v = synth.surveillance_video(600, F)
    say("surveillance 768x576x256", layout)
    model = SpatioTemporalMedian(1, 576, 768, 256, T, 3, 3, layout=layout)
    for f in range(F):
        r = model.push(gpu(v[f]))
        if f in (T, F - 1):
            idx, med = r
            ref = oracle.st_median(v[f - T:f + 1, None], 256, 8, 3, 3)
            assert np.array_equal(med.cpu().numpy(), ref), f
            J = bhw(model.jih, layout)
            assert np.array_equal(J[:, -1, -1], np.cumsum(np.bincount(v[f - T:f + 1].ravel(), minlength=256)))


def test_median_errors():
    ih = ihlib()
    J = torch.zeros((3 * 256, 8, 8), dtype=torch.int32, device=DEV)
    with pytest.raises(ih.IHError):
        ih.ih_local_median(J, 3, 200, 1, 3, 3)                       # plane count mismatch
    with pytest.raises(ih.IHError):
        ih.ih_local_median(J, 3, 256, 0, 3, 3)                       # no frames
    Jh = torch.zeros((8, 8, 3 * 256), dtype=torch.int32, device=DEV)
    img = torch.zeros((3, 8, 8), dtype=torch.uint8, device=DEV)
    with pytest.raises(ih.IHError, match="P <= 512"):
        ih.ih_jih_update(img, None, 256, Jh, layout="hwb")         # 768 planes innermost
    big = torch.zeros((1, 46341, 46341 // 1024), dtype=torch.int32, device=DEV)
    with pytest.raises(ih.IHError, match="int32"):
        ih.ih_local_median(big, 1, 1, 2 * 1024 * 1024, 1, 1)
