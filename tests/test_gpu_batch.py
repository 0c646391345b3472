"""GPU parity of the batched persistent build + search against the oracle."""
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


def make_frames(seed, dtype=np.uint8, n=12, search=True):
    """Uneven frames: sizes from 1x1 to ~300x500, 1-3 channels, 1..64 bins."""
    rng = np.random.default_rng(seed)
    bits = 8 if dtype == np.uint8 else 16
    shapes = [(1, 1), (3, 200), (150, 2), (64, 64), (97, 203), (240, 320), (333, 130), (17, 517),
              (128, 256), (301, 199), (50, 1030), (256, 255)]
    out = []
    for i in range(n):
        H, W = shapes[i % len(shapes)]
        C = int(rng.integers(1, 4)) if i % 3 == 0 else 1
        bins = int(rng.choice([1, 3, 8, 16, 32, 64]))
        img = rng.integers(0, 1 << bits, size=(C, H, W)).astype(dtype)
        if i % 2:
            img = (synth.smooth(rng, H, W, 8)[None].repeat(C, 0) * ((1 << bits) - 1)).astype(dtype)
        fr = dict(np_img=img, img=gpu(img), bins=bins, value_bits=bits)
        if search and H >= 20 and W >= 20:
            th, tw = min(16, H // 2), min(16, W // 2)
            tr, tc = int(rng.integers(0, H - th + 1)), int(rng.integers(0, W - tw + 1))
            origins = synth.grid_origins(tr - 4, tc - 5, 9, 11)          # some outside the frame
            fr.update(np_origins=origins, origins=gpu(origins), win=(th, tw), tmpl_win=(tr, tc, th, tw))
            if i % 4 == 1:   # template descriptor given instead of computed
                fr["np_tmpl"] = oracle.pyramid_desc_direct(img, bins, bits, [[tr, tc, th, tw]], 3)[0]
                fr["tmpl_desc"] = gpu(fr["np_tmpl"])
        out.append(fr)
    return out


def bin_major(batch, i, frames, layout):
    t = batch.ih[i].cpu().numpy()
    return t.transpose(2, 0, 1) if frames[i].get("layout", layout) == "hwb" else t


def check(batch, frames, metric, layout="bhw"):
    for i, fr in enumerate(frames):
        img, bins, bits = fr["np_img"], fr["bins"], fr["value_bits"]
        assert np.array_equal(bin_major(batch, i, frames, layout), oracle.ih(img, bins, bits)), i
        if "origins" not in fr:
            continue
        tr, tc, th, tw = fr["tmpl_win"]
        tmpl = fr.get("np_tmpl")
        if tmpl is None:
            tmpl = oracle.pyramid_desc_direct(img, bins, bits, [[tr, tc, th, tw]], 3)[0]
            assert np.array_equal(batch.tmpl[i].cpu().numpy(), tmpl), i
        od, ob = oracle.match_direct(img, bins, bits, tmpl, th, tw, 3, fr["np_origins"], metric)
        d = batch.dist[i].cpu().numpy().astype(np.float64)
        b = int(batch.best[i].item())
        assert np.array_equal(np.isinf(d), np.isinf(od)), i
        fin = ~np.isinf(od)
        if metric == "chi2":
            assert np.all(np.abs(d[fin] - od[fin]) <= 1e-5 * np.abs(od[fin])), i
            assert abs(od[b] - od[ob]) <= 1e-5 * abs(od[ob]), i
        else:
            assert np.array_equal(d[fin], od[fin].astype(np.float32)), i
            assert b == ob, i


@pytest.mark.parametrize("layout", ["bhw", "hwb"])
@pytest.mark.parametrize("dtype,metric", [(np.uint8, "chi2"), (np.uint16, "l1"), (np.uint8, "pmk")])
def test_batch_matches_oracle(dtype, metric, layout):
    ih = ihlib()
    say("batch", dtype.__name__, metric, layout)
    frames = make_frames(11, dtype)
    batch = ih.Batch(frames, metric, layout=layout)
    batch.run()
    torch.cuda.synchronize()
    check(batch, frames, metric, layout)


def test_batch_mixed_layouts_and_hwb_tiles():
    ih = ihlib()
    frames = make_frames(14, np.uint8, n=12)
    tiles = [ih.TileCfg(16, 16, 64), ih.TileCfg(7, 32, 64), ih.TileCfg(64, 64, 64), ih.TileCfg(1, 16, 64)]
    for i, fr in enumerate(frames):
        if i % 2:
            fr["layout"] = "hwb"
            fr["tile"] = tiles[(i // 2) % len(tiles)]
    batch = ih.Batch(frames, "chi2", layout="bhw")
    batch.run()
    first = [t.clone() for t in batch.ih]
    for rep in range(5):
        batch.run()
    torch.cuda.synchronize()
    for a, b in zip(first, batch.ih):
        assert torch.equal(a, b)
    check(batch, frames, "chi2", "bhw")


def test_batch_tile_shapes_and_repeat():
    ih = ihlib()
    frames = make_frames(12, np.uint8, n=8)
    tiles = [ih.TileCfg(16, 64, 2), ih.TileCfg(7, 128, 8), ih.TileCfg(64, 256, 1), ih.TileCfg(1, 64, 4)]
    for i, fr in enumerate(frames):
        fr["tile"] = tiles[i % len(tiles)]
    batch = ih.Batch(frames, "chi2")
    batch.run()
    first = [t.clone() for t in batch.ih]
    for rep in range(20):
        batch.run()
    torch.cuda.synchronize()
    for a, b in zip(first, batch.ih):
        assert torch.equal(a, b)
    check(batch, frames, "chi2")


@pytest.mark.parametrize("layout", ["bhw", "hwb"])
def test_batch_graph_replays(layout):
    ih = ihlib()
    frames = make_frames(13, np.uint8, n=10)
    batch = ih.Batch(frames, "chi2", layout=layout)
    batch.run()
    torch.cuda.synchronize()
    ref_ih = [t.clone() for t in batch.ih]
    ref_d = [None if d is None else d.clone() for d in batch.dist]
    ref_b = [None if b is None else b.clone() for b in batch.best]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.run()
    for rep in range(4):
        for t in batch.ih:                      # eager work between replays
            t.fill_(-5)
        for d in batch.dist:
            if d is not None:
                d.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(frames)):
            assert torch.equal(batch.ih[i], ref_ih[i]), (rep, i)
            if ref_d[i] is not None:
                assert torch.equal(batch.dist[i], ref_d[i]), (rep, i)
                assert torch.equal(batch.best[i], ref_b[i]), (rep, i)


@pytest.mark.parametrize("layout", ["bhw", "hwb"])
def test_batch_64_graph_replays_parallel_classes(layout):
    """The 64 uneven frames hold two write-out classes in either layout
    (planes innermost staged and in column streams; bin-major tiles and
    strips), whose kernels run as parallel branches forked from and joined
    into the caller's stream.  A graph captured from that stream, replayed
    with eager work in between, reproduces the eager histograms, distances
    and picks bit for bit (the eager batch is checked against the oracle in
    test_batch_64_uneven_frames)."""
    ih = ihlib()
    say("64 uneven frames, graph replays", layout)
    fr4 = synth.config4()
    frames = []
    for f in fr4:
        frames.append(dict(np_img=f.img, img=gpu(f.img), bins=f.bins, value_bits=f.bits,
                           np_origins=f.origins, origins=gpu(f.origins), win=(32, 32), tmpl_win=f.tmpl_win))
    batch = ih.Batch(frames, "chi2", layout=layout)
    batch.run()
    torch.cuda.synchronize()
    ref_ih = [t.clone() for t in batch.ih]
    ref_d = [d.clone() for d in batch.dist]
    ref_b = [b.clone() for b in batch.best]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.run()
    for rep in range(3):
        for t in batch.ih:                      # eager work between replays
            t.fill_(-5)
        for d in batch.dist:
            d.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(frames)):
            assert torch.equal(batch.ih[i], ref_ih[i]), (rep, i)
            assert torch.equal(batch.dist[i], ref_d[i]), (rep, i)
            assert torch.equal(batch.best[i], ref_b[i]), (rep, i)


@pytest.mark.parametrize("layout", ["bhw", "hwb"])
def test_batch_64_uneven_frames(layout):
    ih = ihlib()
    say("64 uneven frames, 4096 candidates each", layout)
    fr4 = synth.config4()
    frames = []
    for f in fr4:
        frames.append(dict(np_img=f.img, img=gpu(f.img), bins=f.bins, value_bits=f.bits,
                           np_origins=f.origins, origins=gpu(f.origins), win=(32, 32), tmpl_win=f.tmpl_win))
    batch = ih.Batch(frames, "chi2", layout=layout)
    batch.run()
    torch.cuda.synchronize()
    for i, f in enumerate(fr4):
        b = int(batch.best[i].item())
        assert tuple(f.origins[b]) == tuple(f.tmpl_win[:2]), i       # D = 0 at the template's own origin
        assert float(batch.dist[i][b]) == 0.0
    for i in (0, 7, 31, 63):
        say("frame", i, fr4[i].img.shape, fr4[i].bins)
        f = fr4[i]
        assert np.array_equal(bin_major(batch, i, frames, layout), oracle.ih(f.img, f.bins, f.bits)), i
        tmpl = oracle.pyramid_desc_direct(f.img, f.bins, f.bits, [f.tmpl_win], 3)[0]
        od, ob = oracle.match_direct(f.img, f.bins, f.bits, tmpl, 32, 32, 3, f.origins, "chi2")
        d = batch.dist[i].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(d - od) <= 1e-5 * np.abs(od)), i


@pytest.mark.parametrize("layout", ["bhw", "hwb", "any"])
def test_batch_tile_per_bin_class(layout):
    """tune_batch_classes gives every frame a candidate shape (and with "any"
    a layout), one per bin count, never slower (as timed) than the uniform
    shape it starts from; the batch built with those choices matches the
    oracle."""
    ih = ihlib()
    from paper_1711_01656_amd import tune
    frames = make_frames(21, np.uint8, n=10)
    say("tune per class", layout)
    tiles, by_bins, best_ms, uniform_ms = tune.tune_batch_classes(frames, "chi2", layout=layout, reps=1)
    lays = ("bhw", "hwb") if layout == "any" else (layout,)
    cands = {(l, repr(c)) for l in lays for c in tune.batch_candidates(l)}
    assert len(tiles) == len(frames)
    assert set(by_bins) == {int(f["bins"]) for f in frames}
    for fr, (fl, t) in zip(frames, tiles):
        assert (fl, repr(t)) in cands and (fl, t) == by_bins[int(fr["bins"])]
    assert best_ms <= uniform_ms
    for fr, (fl, t) in zip(frames, tiles):
        fr["layout"], fr["tile"] = fl, t
    batch = ih.Batch(frames, "chi2", layout="bhw")
    batch.run()
    torch.cuda.synchronize()
    check(batch, frames, "chi2", "bhw")
