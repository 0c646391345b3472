"""Host-side logic of the tracker and the proposal binding (no GPU)."""
import numpy as np

from paper_1711_01656_amd import proposal as lp
from paper_1711_01656_amd import tracker as trk
from synth.video import Video, render


def test_label_offset_round_trip():
    dy, dx = np.meshgrid(np.arange(-32, 33), np.arange(-32, 33), indexing="ij")
    lab = lp.label_of(dy.ravel(), dx.ravel())
    assert np.array_equal(lab, np.arange(4225))
    ry, rx = lp.offset_of(lab)
    assert np.array_equal(ry, dy.ravel()) and np.array_equal(rx, dx.ravel())


def test_parameter_layout():
    assert lp.N_PARAMS == 32 * 63 + 32 + 2 * (32 * 288 + 32) + 32 + 1
    p = lp.init_params(0)
    assert set(p) == {n for n, _ in lp.PARAM_LAYOUT}
    assert all(p[n].shape == s for n, s in lp.PARAM_LAYOUT)


def test_distance_prior_ranks_nearest_offsets_first():
    prior = trk.distance_prior().numpy().ravel()
    order = np.lexsort((np.arange(4225), -prior))[:64]
    dy, dx = lp.offset_of(order)
    d2 = dy ** 2 + dx ** 2
    assert d2.max() <= 20 and d2[0] == 0 and np.all(np.diff(d2) >= 0)


def test_samples_from_track():
    t = trk.Track(origins=np.array([[10, 20], [12, 18], [12, 18], [60, 18]]), dists=np.array([0, 1.0, 2.0, 3.0]),
                  fallback=np.zeros(4, bool))
    s = trk.samples_from_track(t, (9, 11), frame0=100)
    # the jump of 48 rows leaves the search range and is dropped
    assert s.frame.tolist() == [101, 102]
    assert s.center.tolist() == [[14, 25], [16, 23]]
    assert s.offset.tolist() == [[2, -2], [0, 0]]


def test_video_is_seeded_and_target_moves_within_range():
    a, b = Video(5, 180, 320, 12), Video(5, 180, 320, 12)
    fa, fb = render(a, threads=2), render(b, threads=2)
    assert fa.shape == (12, 7, 180, 320) and np.array_equal(fa, fb)
    c = np.array([a.target_box(t)[:2] for t in range(12)])
    assert np.abs(np.diff(c, axis=0)).max() <= 9
    r, q, h, w = a.target_box(0)
    assert 21 <= h <= 81 and 21 <= w <= 81 and r >= 0 and q >= 0 and r + h <= 180 and q + w <= 320


def test_coarser_pyramid_distances_are_lower_bounds():
    """Reading of the bounded search: chi-square and L1 never rise when cells
    merge, and with Eq. 2.24's weights each added level raises the distance by
    a non-negative combination of level-sum differences, so the oracle's
    distances satisfy D_1 <= D_2 <= D_3 <= D_4 for every candidate of random
    and structured scenes, each strictly somewhere (the bounds are not
    trivially tight)."""
    import oracle
    rng = np.random.default_rng(41)
    for trial in range(6):
        H, W = 40 + 7 * trial, 55 + 5 * trial
        img = rng.integers(0, 256, size=(2, H, W)).astype(np.uint8)
        if trial % 2:
            img[:, : H // 2] //= 4                      # two textures
        h, w = 12 + trial, 16
        tr, tc = int(rng.integers(0, H - h)), int(rng.integers(0, W - w))
        ys, xs = np.meshgrid(np.arange(-3, H - h + 3), np.arange(-3, W - w + 3), indexing="ij")
        origins = np.stack([ys.ravel(), xs.ravel()], 1).astype(np.int32)
        for metric in ("chi2", "l1"):
            full = oracle.pyramid_desc_direct(img, 8, 8, np.array([[tr, tc, h, w]], np.int32), 4)[0]
            d = []
            for lv in (1, 2, 3, 4):
                t = oracle.pyramid_desc_direct(img, 8, 8, np.array([[tr, tc, h, w]], np.int32), lv)[0]
                assert np.array_equal(t.ravel(), full.ravel()[: t.size])   # coarser levels lead the descriptor
                d.append(oracle.match_direct(img, 8, 8, t, h, w, lv, origins, metric)[0])
            fin = np.isfinite(d[-1])
            for lo, hi in zip(d[:-1], d[1:]):
                assert np.array_equal(fin, np.isfinite(lo))
                assert np.all(lo[fin] <= hi[fin] * (1 + 1e-12) + 1e-12), (trial, metric)
                assert np.any(lo[fin] < hi[fin] * (1 - 1e-6))
