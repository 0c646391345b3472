"""Pins for the oracle's FG/BG colour likelihood (Eq. 2.18-2.21), moment
integral images and CAMSHIFT (Alg. 1): numpy joint histograms and
floating-point rounding for the likelihood, cumulative sums for the moment
images, and for CAMSHIFT closed-form fixed points (a single bright pixel, a
symmetric blob), degenerate maps and the fixed-point property of its result."""
import numpy as np
import pytest

import oracle


def joint_bins(rgb):
    return ((rgb[0].astype(np.int64) >> 3) * 32 + (rgb[1] >> 3)) * 32 + (rgb[2] >> 3)


def test_likelihood_matches_numpy_histograms():
    rng = np.random.default_rng(1)
    H, W = 60, 80
    rgb = rng.integers(0, 64, size=(3, H, W)).astype(np.uint8) * 4      # few colours, many collisions
    fg = np.array([20, 30, 40, 55], np.int32)
    bg = np.array([10, 15, 52, 72], np.int32)
    q, L = oracle.color_likelihood(rgb, fg, bg)
    b = joint_bins(rgb)
    in_fg = np.zeros((H, W), bool)
    in_fg[20:40, 30:55] = True
    in_bg = np.zeros((H, W), bool)
    in_bg[10:52, 15:72] = True
    in_bg &= ~in_fg
    hf = np.bincount(b[in_fg], minlength=32768).astype(np.float64)
    hb = np.bincount(b[in_bg], minlength=32768).astype(np.float64)
    t = hf[b] + hb[b]
    Lref = np.where(t > 0, hf[b] / np.maximum(t, 1), 0.0)
    np.testing.assert_allclose(L, Lref, rtol=0, atol=1e-15)
    assert np.array_equal(q, np.floor(255 * Lref + 0.5).astype(np.uint8))
    assert (L[in_fg] > 0).all()                      # every FG colour has FG mass


def test_likelihood_hand_example():
    """2 x 3 image; FG = column 0, BG = the whole image minus column 0.
    Colours: A at (0,0), (0,1); B at (1,0); C at (1,1), (0,2), (1,2)."""
    A, B, C = (200, 10, 10), (10, 200, 10), (10, 10, 200)
    img = [[A, A, C], [B, C, C]]
    rgb = np.array(img, np.uint8).transpose(2, 0, 1).copy()
    q, L = oracle.color_likelihood(rgb, [0, 0, 2, 1], [0, 0, 2, 3])
    # A: 1 FG, 1 BG -> 0.5 (q = 128, half rounds up); B: 1 FG -> 1; C: 3 BG -> 0
    assert L.tolist() == [[0.5, 0.5, 0.0], [1.0, 0.0, 0.0]]
    assert q.tolist() == [[128, 128, 0], [255, 0, 0]]


def test_moment_images_are_cumsums():
    rng = np.random.default_rng(2)
    q = rng.integers(0, 256, size=(37, 53)).astype(np.uint8)
    S, Sx, Sy = oracle.moment_images(q)
    v = q.astype(np.int64)
    r = np.arange(37)[:, None]
    c = np.arange(53)[None, :]
    assert np.array_equal(S, v.cumsum(0).cumsum(1))
    assert np.array_equal(Sx, (v * r).cumsum(0).cumsum(1))
    assert np.array_equal(Sy, (v * c).cumsum(0).cumsum(1))


def test_camshift_single_pixel():
    q = np.zeros((50, 60), np.uint8)
    q[23, 41] = 200
    cen, it = oracle.camshift(q, [[20.0, 38.0], [27.4, 44.6]], 11, 11)
    assert np.array_equal(cen, [[23.0, 41.0], [23.0, 41.0]])
    assert (it == 2).all()                           # one move, then a move of 0


def test_camshift_symmetric_blob_and_fixed_point():
    H, W = 120, 140
    r = np.arange(H)[:, None]
    c = np.arange(W)[None, :]
    q = np.where((r - 60.0) ** 2 + (c - 75.0) ** 2 <= 15 ** 2, 180, 0).astype(np.uint8)
    rng = np.random.default_rng(3)
    starts = np.stack([60 + rng.uniform(-12, 12, 50), 75 + rng.uniform(-12, 12, 50)], 1)
    cen, it = oracle.camshift(q, starts, 41, 41, delta=0.01, max_iter=50)
    np.testing.assert_allclose(cen, np.tile([60.0, 75.0], (50, 1)), atol=0.05)
    # fixed point: the centroid of the window placed at the result moves it by < delta
    q2 = np.random.default_rng(4).integers(0, 256, size=(H, W)).astype(np.uint8)
    cen2, it2 = oracle.camshift(q2, starts, 31, 25, delta=0.25, max_iter=100)
    for (cr, cc), n in zip(cen2, it2):
        assert n < 100
        r0 = min(max(int(np.floor(cr - 15 + 0.5)), 0), H - 31)
        c0 = min(max(int(np.floor(cc - 12 + 0.5)), 0), W - 25)
        win = q2[r0:r0 + 31, c0:c0 + 25].astype(np.float64)
        m = win.sum()
        nr = (win * np.arange(r0, r0 + 31)[:, None]).sum() / m
        nc = (win * np.arange(c0, c0 + 25)[None, :]).sum() / m
        assert (nr - cr) ** 2 + (nc - cc) ** 2 < 0.25 ** 2


def test_camshift_degenerate():
    q = np.zeros((20, 20), np.uint8)
    cen, it = oracle.camshift(q, [[5.5, 6.25]], 5, 5)
    assert cen.tolist() == [[5.5, 6.25]] and it.tolist() == [1]
    q[10, 10] = 9
    cen, it = oracle.camshift(q, [[3.0, 3.0]], 5, 5, max_iter=0)
    assert cen.tolist() == [[3.0, 3.0]] and it.tolist() == [0]
    with pytest.raises(RuntimeError):
        oracle.camshift(q, [[3.0, 3.0]], 21, 5)        # window taller than the map
