"""The seeded input generators: shapes, dtypes, determinism, value ranges."""
import numpy as np

import synth


def test_config1_shapes_and_determinism():
    a = synth.config1()
    b = synth.config1()
    assert a.img.shape == (1, 480, 640) and a.img.dtype == np.uint8
    assert np.array_equal(a.img, b.img) and np.array_equal(a.rects, b.rects)
    h = a.rects[:, 2] - a.rects[:, 0]
    w = a.rects[:, 3] - a.rects[:, 1]
    assert a.rects.shape == (10_000, 4)
    assert h.min() >= 4 and h.max() <= 200 and w.min() >= 4 and w.max() <= 200
    assert a.rects[:, 0].min() >= 0 and a.rects[:, 2].max() <= 480 and a.rects[:, 3].max() <= 640
    assert a.img.std() > 20          # textured, not flat


def test_config2_channels():
    w = synth.config2(scale=0.25, n_windows=1000)
    assert w.img.shape == (7, 270, 480) and w.img.dtype == np.uint8
    assert w.P == 112 and w.moments
    assert set(np.unique(w.img[6])) <= {0, 255}
    hw = w.windows[:, 2:] - w.windows[:, :2]
    assert hw.min() >= 16 and hw.max() <= 256


def test_config3_small_scale():
    w = synth.config3(scale=1 / 16, n_rects=100)
    assert w.img.dtype == np.uint16 and w.img.shape == (1, 512, 512)
    assert w.origins.shape == (129 * 129, 2)
    tr, tc, th, tw = w.tmpl_win
    assert tr - 64 >= 0 and tc - 64 >= 0 and tr + 64 + th <= 512 and tc + 64 + tw <= 512
    assert w.img.max() >= 50000      # blobs present


def test_config4_frames():
    fr = synth.config4(n_frames=4, scale=0.25)
    for f in fr:
        H, W = f.img.shape[1:]
        assert f.bins in (8, 16, 32, 64)
        assert f.origins.shape == (4096, 2)
        assert f.origins[:, 0].min() >= 0 and f.origins[:, 0].max() + 32 <= H
        assert f.origins[:, 1].min() >= 0 and f.origins[:, 1].max() + 32 <= W
