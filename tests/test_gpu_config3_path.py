"""GPU parity of the exact kernels the 8192x8192 u16 (64 bins) workload times:
the planes-innermost u16 builds with 32- and 64-column staged tiles, and the
1M rectangle queries and 129x129 pyramid search on the planes-innermost
17 GB tensor, against the oracle (bit-exact; chi-square within 1e-5)."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# tile shapes the benchmark runs on this workload (tile_h, tile_w, planes_per_wave)
BENCH_TILES = [(128, 32, 64), (128, 64, 64)]


def ihlib():
    import paper_1711_01656_amd as ih
    return ih


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(*a):
    print(*a, flush=True)


def aerial_u16(seed, H, W):
    """A ragged u16 frame with the 8192^2 workload's value structure."""
    return synth.aerial_u16(seed, H, W, 200, seed + 1)[0][None]


@pytest.mark.parametrize("tile", BENCH_TILES)
def test_u16_hwb_bench_tiles_ragged_full(tile):
    """1000 x 3000 u16, 64 bins: 1000 = 7 * 128 + 104 rows and 3000 columns
    leave a ragged last tile in both directions."""
    ih = ihlib()
    img = aerial_u16(31, 1000, 3000)
    cfg = ih.TileCfg(*tile)
    say("u16 hwb", cfg)
    out = ih.ih_build(gpu(img), 64, 16, cfg=cfg, layout="hwb")
    ref = oracle.ih(img, 64, 16)
    assert np.array_equal(out.permute(2, 0, 1).cpu().numpy(), ref)


@pytest.mark.parametrize("tile", BENCH_TILES)
def test_config3_hwb_build_sampled(tile):
    ih = ihlib()
    w = synth.config3(n_rects=1)
    cfg = ih.TileCfg(*tile)
    say("8192^2 u16 x 64 bins, planes innermost", cfg)
    out = ih.ih_build(gpu(w.img), w.bins, w.bits, cfg=cfg, layout="hwb")
    torch.cuda.synchronize()
    idx = oracle.plane_index(w.img, w.bins, w.bits)
    counts = np.bincount(idx.ravel(), minlength=w.P)
    assert np.array_equal(out[-1, -1, :].cpu().numpy(), counts)
    # every pixel's histogram sums to its (r+1)(c+1) area: checked on the last
    # row and the last column of the frame
    W, H = w.W, w.H
    assert bool((out[-1].sum(1, dtype=torch.int64) == torch.arange(1, W + 1, device=DEV) * H).all())
    assert bool((out[:, -1].sum(1, dtype=torch.int64) == torch.arange(1, H + 1, device=DEV) * W).all())
    for p in (0, 17, 40, 63):
        say("plane", p)
        got = out[:, :, p].contiguous().cpu().numpy()
        assert np.array_equal(got, oracle.ih_plane(w.img, w.bins, w.bits, p)), p
    del out
    torch.cuda.empty_cache()


def test_config3_hwb_queries_and_search_sampled():
    ih = ihlib()
    w = synth.config3()
    cfg = ih.TileCfg(*BENCH_TILES[1])
    say("8192^2 planes innermost: 1M rects, 129x129 search")
    H_ = ih.ih_build(gpu(w.img), w.bins, w.bits, cfg=cfg, layout="hwb")
    out = ih.ih_query_rect(H_, gpu(w.rects), layout="hwb")
    idx = np.random.default_rng(7).choice(len(w.rects), 3000, replace=False)
    ref = oracle.query_rect_direct(w.img, w.bins, w.bits, w.rects[idx])
    assert np.array_equal(out[torch.from_numpy(idx).to(DEV)].cpu().numpy(), ref)
    area = (w.rects[:, 2] - w.rects[:, 0]).astype(np.int64) * (w.rects[:, 3] - w.rects[:, 1])
    assert np.array_equal(out.sum(1, dtype=torch.int64).cpu().numpy(), area)
    tmpl = oracle.pyramid_desc_direct(w.img, w.bins, w.bits, [w.tmpl_win], 3)[0]
    gd = ih.ih_pyramid_desc(H_, gpu(np.array([w.tmpl_win], np.int32)), 3, layout="hwb").cpu().numpy()[0]
    assert np.array_equal(gd, tmpl)
    d, b = ih.ih_match_candidates(H_, gpu(tmpl), 32, 32, gpu(w.origins), 3, "chi2", layout="hwb")
    od, ob = oracle.match_direct(w.img, w.bins, w.bits, tmpl, 32, 32, 3, w.origins, "chi2")
    d = d.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(d - od) <= 1e-5 * np.abs(od))
    assert int(b.item()) == ob and tuple(w.origins[ob]) == w.tmpl_win[:2]
    del H_, out
    torch.cuda.empty_cache()
