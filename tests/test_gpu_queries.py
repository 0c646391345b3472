"""GPU parity of the region queries, pyramid descriptors and candidate search."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def ihlib():
    import paper_1711_01656_amd as ih
    return ih


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(*a):
    print(*a, flush=True)


def rand_rects(seed, H, W, n, lo=1, hi=None):
    hi = hi or max(H, W)
    return synth.rects_uniform(seed, H, W, n, lo, hi)


@pytest.fixture(scope="module", params=["bhw", "hwb"])
def scene(request):
    layout = request.param
    img = synth.feature_channels(77, 123, 301)[:3]          # 3 channels
    bins = 8
    ih = ihlib()
    t = gpu(img)
    H_, mx, my = ih.ih_build(t, bins, moments=True, layout=layout)
    ref = oracle.ih(img, bins, 8)
    omx, omy = oracle.moments(img, bins, 8)
    return dict(img=img, bins=bins, t=t, H=H_, mx=mx, my=my, ref=ref, omx=omx, omy=omy, C=3, L=layout)


def test_query_rect_exact(scene):
    ih = ihlib()
    rects = rand_rects(1, 123, 301, 5000)
    extra = np.array([[0, 0, 123, 301], [5, 5, 5, 9], [0, 0, 1, 1], [122, 300, 123, 301],
                      [-1, 0, 4, 4], [0, 0, 124, 3], [10, 10, 9, 12], [3, 7, 3, 7]], np.int32)
    rects = np.concatenate([rects, extra])
    out = ih.ih_query_rect(scene["H"], gpu(rects), layout=scene["L"]).cpu().numpy()
    assert np.array_equal(out, oracle.query_rect(scene["ref"], rects))
    assert np.array_equal(out[:5000], oracle.query_rect_direct(scene["img"], scene["bins"], 8, rects[:5000]))


def test_query_rect_empty_batch(scene):
    ih = ihlib()
    out = ih.ih_query_rect(scene["H"], torch.empty((0, 4), dtype=torch.int32, device=DEV), layout=scene["L"])
    assert out.shape == (0, 24)


def test_query_weighted_bit_exact_and_tolerance(scene):
    ih = ihlib()
    rects = rand_rects(2, 123, 301, 3000, 1, 123)
    extra = np.array([[0, 0, 1, 1], [0, 0, 123, 301], [4, 4, 4, 10], [0, 0, 124, 2], [7, 3, 9, 4]], np.int32)
    rects = np.concatenate([rects, extra])
    for l1 in (False, True):
        say("weighted l1 =", l1)
        out = ih.ih_query_weighted(scene["H"], scene["mx"], scene["my"], scene["C"], gpu(rects),
                                   l1_normalize=l1, layout=scene["L"]).cpu().numpy()
        _, ref = oracle.weighted_swih(scene["ref"], scene["omx"], scene["omy"], scene["C"], rects, l1norm=l1)
        assert np.array_equal(np.isnan(out), np.isnan(ref))
        ok = ~np.isnan(ref)
        assert np.array_equal(out[ok], ref[ok])              # same integer numerator, same rounding
        bf = oracle.weighted_bruteforce(scene["img"], scene["bins"], 8, rects[:600], l1norm=l1)
        o = out[:600].astype(np.float64)
        assert np.all(np.abs(o - bf) <= 1e-5 * np.abs(bf))    # <= 1e-5 relative to FP64
        assert np.all((o == 0) == (bf == 0))


def test_query_weighted_wrap_guard():
    ih = ihlib()
    img = np.zeros((1, 64, 64), np.uint8)
    H_, mx, my = ih.ih_build(gpu(img), 2, moments=True)
    out = ih.ih_query_weighted(H_, mx, my, 1, gpu(np.array([[0, 0, 64, 64]], np.int32))).cpu().numpy()
    assert np.all(np.isfinite(out))
    # a window whose moment sums could pass 2^32 is refused with NaN
    img = np.zeros((1, 2048, 2048), np.uint8)
    H_, mx, my = ih.ih_build(gpu(img), 2, moments=True)
    out = ih.ih_query_weighted(H_, mx, my, 1, gpu(np.array([[0, 0, 2048, 2048], [0, 0, 1024, 1024]],
                                                           np.int32))).cpu().numpy()
    assert np.all(np.isnan(out[0])) and np.all(np.isfinite(out[1]))


def test_pyramid_desc_exact(scene):
    ih = ihlib()
    rng = np.random.default_rng(3)
    wins = []
    for _ in range(700):
        h, w = int(rng.integers(1, 90)), int(rng.integers(1, 120))
        wins.append([int(rng.integers(0, 123 - h + 1)), int(rng.integers(0, 301 - w + 1)), h, w])
    wins += [[0, 0, 123, 301], [-1, 0, 4, 4], [0, 0, 0, 3], [120, 298, 4, 4]]
    wins = np.array(wins, np.int32)
    for levels in (1, 2, 3, 4):
        say("pyramid levels", levels)
        out = ih.ih_pyramid_desc(scene["H"], gpu(wins), levels, layout=scene["L"]).cpu().numpy()
        assert np.array_equal(out, oracle.pyramid_desc(scene["ref"], wins, levels))


@pytest.mark.parametrize("metric", ["chi2", "l1", "pmk"])
@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_match_candidates(scene, metric, levels):
    ih = ihlib()
    say("match", metric, levels)
    img, bins = scene["img"], scene["bins"]
    tr, tc, th, tw = 40, 120, 24, 20
    tmpl = oracle.pyramid_desc_direct(img, bins, 8, [[tr, tc, th, tw]], levels)[0]
    origins = synth.grid_origins(tr - 45, tc - 30, 91, 61)   # partly outside the frame
    d, b = ih.ih_match_candidates(scene["H"], gpu(tmpl), th, tw, gpu(origins), levels, metric,
                                  layout=scene["L"])
    d = d.cpu().numpy().astype(np.float64)
    b = int(b.item())
    od, ob = oracle.match_direct(img, bins, 8, tmpl, th, tw, levels, origins, metric)
    assert np.array_equal(np.isinf(d), np.isinf(od))
    fin = ~np.isinf(od)
    if metric == "chi2":
        assert np.all(np.abs(d[fin] - od[fin]) <= 1e-5 * np.abs(od[fin]))
        assert abs(od[b] - od[ob]) <= 1e-5 * abs(od[ob])      # tie-tolerant argmin
    else:
        assert np.array_equal(d[fin], od[fin].astype(np.float32).astype(np.float64))
        assert b == ob
    assert tuple(origins[ob]) == (tr, tc)


def test_match_no_candidate_inside(scene):
    ih = ihlib()
    tmpl = np.zeros((21, 24), np.int32)
    origins = np.array([[-5, -5], [200, 0]], np.int32)
    d, b = ih.ih_match_candidates(scene["H"], gpu(tmpl), 8, 8, gpu(origins), 3, "chi2", layout=scene["L"])
    assert int(b.item()) == -1 and np.all(np.isinf(d.cpu().numpy()))


@pytest.mark.parametrize("layout", ["bhw", "hwb"])
def test_config1_rect_queries_full(layout):
    ih = ihlib()
    w = synth.config1()
    H_ = ih.ih_build(gpu(w.img), w.bins, layout=layout)
    out = ih.ih_query_rect(H_, gpu(w.rects), layout=layout).cpu().numpy()
    assert np.array_equal(out, oracle.query_rect_direct(w.img, w.bins, w.bits, w.rects))


@pytest.mark.parametrize("layout", ["bhw", "hwb"])
def test_config2_weighted_full_sampled(layout):
    ih = ihlib()
    w = synth.config2()
    say("config 1920x1080 weighted 100k", layout)
    H_, mx, my = ih.ih_build(gpu(w.img), w.bins, moments=True, layout=layout)
    out = ih.ih_query_weighted(H_, mx, my, w.C, gpu(w.windows), layout=layout).cpu().numpy()
    assert np.all(np.isfinite(out))
    idx = np.random.default_rng(5).choice(len(w.windows), 300, replace=False)
    bf = oracle.weighted_bruteforce(w.img, w.bins, w.bits, w.windows[idx])
    o = out[idx].astype(np.float64)
    assert np.all(np.abs(o - bf) <= 1e-5 * np.abs(bf))
    assert np.all((o == 0) == (bf == 0))
    # per-channel totals: the closed form of the Manhattan weights
    h = (w.windows[:, 2] - w.windows[:, 0]).astype(np.float64)
    ww = (w.windows[:, 3] - w.windows[:, 1]).astype(np.float64)
    tot = (2 * h * ww * h * ww - ww * ww * 2 * np.floor(h * h / 4) - h * h * 2 * np.floor(ww * ww / 4)) / (2 * h * ww)
    for ch in range(w.C):
        np.testing.assert_allclose(out[:, ch * 16:(ch + 1) * 16].astype(np.float64).sum(1), tot, rtol=1e-5)


def test_config3_queries_and_match_sampled():
    ih = ihlib()
    w = synth.config3()
    say("config 8192^2: build, 1M rects, 129x129 match")
    t = gpu(w.img)
    H_ = ih.ih_build(t, w.bins, w.bits)
    out = ih.ih_query_rect(H_, gpu(w.rects))
    idx = np.random.default_rng(6).choice(len(w.rects), 3000, replace=False)
    ref = oracle.query_rect_direct(w.img, w.bins, w.bits, w.rects[idx])
    assert np.array_equal(out[torch.from_numpy(idx).to(DEV)].cpu().numpy(), ref)
    area = (w.rects[:, 2] - w.rects[:, 0]).astype(np.int64) * (w.rects[:, 3] - w.rects[:, 1])
    assert np.array_equal(out.sum(1, dtype=torch.int64).cpu().numpy(), area)
    tmpl = oracle.pyramid_desc_direct(w.img, w.bins, w.bits, [w.tmpl_win], 3)[0]
    d, b = ih.ih_match_candidates(H_, gpu(tmpl), 32, 32, gpu(w.origins), 3, "chi2")
    od, ob = oracle.match_direct(w.img, w.bins, w.bits, tmpl, 32, 32, 3, w.origins, "chi2")
    d = d.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(d - od) <= 1e-5 * np.abs(od))
    assert int(b.item()) == ob and tuple(w.origins[ob]) == w.tmpl_win[:2]
    gd = ih.ih_pyramid_desc(H_, gpu(np.array([w.tmpl_win], np.int32)), 3).cpu().numpy()[0]
    assert np.array_equal(gd, tmpl)
    del H_, out
    torch.cuda.empty_cache()
