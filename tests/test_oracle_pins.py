"""Pins for the CPU oracle: each check ties it to something other than itself
(brute force, library routines on special cases, closed forms, invariants and a
hand-worked fixture), so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them."""
import itertools

import numpy as np
import pytest

import oracle


def rand_img(rng, C, H, W, bits):
    dt = np.uint8 if bits <= 8 else np.uint16
    return rng.integers(0, 1 << bits, size=(C, H, W)).astype(dt)


def onehot(img, bins, bits):
    """Per-plane indicator arrays, built with numpy's digitize over equal-width edges."""
    C, H, W = img.shape
    edges = np.arange(1, bins) * (1 << bits) / bins  # interior edges of equal-width bins
    planes = []
    for ch in range(C):
        b = np.digitize(img[ch].astype(np.float64), edges, right=False)
        for k in range(bins):
            planes.append((b == k).astype(np.int64))
    return np.stack(planes)


# --------------------------------------------------------------------------- #
# Binning (Eq. 2.15's Q with equal-width bins)                                 #
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("bins,bits", [(1, 8), (2, 8), (3, 8), (7, 8), (32, 8), (64, 16), (5, 16), (256, 8)])
def test_binning_equal_width(bins, bits):
    vals = np.arange(1 << bits, dtype=np.uint16 if bits > 8 else np.uint8)
    idx = oracle.plane_index(vals.reshape(1, 1, -1), bins, bits).ravel()
    assert idx[0] == 0 and idx[-1] == bins - 1
    assert np.all(np.diff(idx) >= 0) and np.all(np.diff(idx) <= 1)
    counts = np.bincount(idx, minlength=bins)
    assert counts.max() - counts.min() <= 1          # equal widths up to one value
    assert counts.sum() == 1 << bits


def test_binning_matches_digitize():
    rng = np.random.default_rng(0)
    for bins, bits in [(3, 8), (10, 8), (64, 16), (16, 8)]:
        img = rand_img(rng, 1, 9, 11, bits)
        idx = oracle.plane_index(img, bins, bits)[0]
        oh = onehot(img, bins, bits)
        assert np.array_equal(oh.argmax(0), idx)


def test_binning_power_of_two_is_shift():
    rng = np.random.default_rng(1)
    img = rand_img(rng, 1, 20, 20, 16)
    assert np.array_equal(oracle.plane_index(img, 64, 16)[0], img[0] >> 10)


# --------------------------------------------------------------------------- #
# Integral histogram (Eq. 2.15, Alg. 5)                                        #
# --------------------------------------------------------------------------- #
TINY = [(1, 1), (1, 7), (5, 1), (3, 4), (7, 9), (16, 16), (13, 5)]


@pytest.mark.parametrize("H,W", TINY)
@pytest.mark.parametrize("C,bins,bits", [(1, 1, 8), (1, 4, 8), (2, 3, 8), (1, 8, 16), (3, 5, 16)])
def test_recurrence_equals_double_sum(H, W, C, bins, bits):
    img = rand_img(np.random.default_rng(H * 100 + W + bins), C, H, W, bits)
    assert np.array_equal(oracle.ih(img, bins, bits), oracle.ih_bruteforce(img, bins, bits))


@pytest.mark.parametrize("H,W,C,bins,bits", [(31, 47, 1, 8, 8), (64, 97, 2, 16, 8), (29, 61, 1, 64, 16)])
def test_ih_equals_numpy_cumsum(H, W, C, bins, bits):
    img = rand_img(np.random.default_rng(7), C, H, W, bits)
    ref = onehot(img, bins, bits).cumsum(1).cumsum(2)
    assert np.array_equal(oracle.ih(img, bins, bits), ref)


def test_ih_invariants():
    rng = np.random.default_rng(3)
    C, H, W, bins, bits = 2, 37, 53, 12, 8
    img = rand_img(rng, C, H, W, bits)
    ih = oracle.ih(img, bins, bits).astype(np.int64)
    # last entry equals the per-bin pixel count
    idx = oracle.plane_index(img, bins, bits)
    assert np.array_equal(ih[:, -1, -1], np.bincount(idx.ravel(), minlength=C * bins))
    # the sum over bins equals the area, per channel
    r = np.arange(1, H + 1)[:, None]
    c = np.arange(1, W + 1)[None, :]
    assert np.array_equal(ih.sum(0), C * r * c)
    for ch in range(C):
        assert np.array_equal(ih[ch * bins:(ch + 1) * bins].sum(0), r * c)
    # monotone non-decreasing along rows and columns
    assert np.all(np.diff(ih, axis=1) >= 0) and np.all(np.diff(ih, axis=2) >= 0)


def test_ih_special_cases():
    H, W = 9, 14
    r = np.arange(1, H + 1)[:, None]
    c = np.arange(1, W + 1)[None, :]
    rng = np.random.default_rng(4)
    # one bin: (r+1)(c+1)
    img = rand_img(rng, 1, H, W, 8)
    assert np.array_equal(oracle.ih(img, 1, 8)[0], r * c)
    # constant image: one plane carries the area, the others are zero
    const = np.full((1, H, W), 77, np.uint8)
    ih = oracle.ih(const, 8, 8)
    k = 77 * 8 // 256
    assert np.array_equal(ih[k], r * c)
    assert not np.any(np.delete(ih, k, axis=0))
    # single impulse: a step at the impulse position
    imp = np.zeros((1, H, W), np.uint8)
    imp[0, 4, 6] = 255
    ih = oracle.ih(imp, 2, 8)
    step = np.zeros((H, W), np.int64)
    step[4:, 6:] = 1
    assert np.array_equal(ih[1], step)
    assert np.array_equal(ih[0], r * c - step)


def test_ih_transpose_symmetry():
    img = rand_img(np.random.default_rng(5), 1, 23, 31, 8)
    a = oracle.ih(img, 6, 8)
    b = oracle.ih(np.ascontiguousarray(img.transpose(0, 2, 1)), 6, 8)
    assert np.array_equal(a.transpose(0, 2, 1), b)


def test_ih_golden(golden):
    g = golden("ih_3x4_2bins.txt")
    img = np.array(g["image"], dtype=np.uint8)[None]
    ih = oracle.ih(img, 2, 8)
    assert np.array_equal(ih[0], np.array(g["ih_plane0"], int))
    assert np.array_equal(ih[1], np.array(g["ih_plane1"], int))
    out = oracle.query_rect(ih, [list(map(int, g["rect"][0]))])
    assert out[0].tolist() == [int(v) for v in g["rect_hist"][0]]


def test_ih_plane_streaming_equals_full():
    img = rand_img(np.random.default_rng(6), 2, 19, 27, 16)
    full = oracle.ih(img, 8, 16)
    for p in range(16):
        assert np.array_equal(oracle.ih_plane(img, 8, 16, p), full[p])


def test_value_range_check():
    img = np.array([[[0, 255]]], np.uint8)
    assert oracle.check_values(img, 8)
    assert not oracle.check_values(img, 7)


# --------------------------------------------------------------------------- #
# Coordinate moments (Eq. 3.4 weights spanned by 1, row, column)               #
# --------------------------------------------------------------------------- #
def test_moments_equal_numpy_cumsum():
    rng = np.random.default_rng(8)
    C, H, W, bins = 2, 21, 34, 5
    img = rand_img(rng, C, H, W, 8)
    oh = onehot(img, bins, 8)
    rr = np.arange(H)[None, :, None]
    cc = np.arange(W)[None, None, :]
    mx, my = oracle.moments(img, bins, 8)
    assert np.array_equal(mx, (oh * rr).cumsum(1).cumsum(2))
    assert np.array_equal(my, (oh * cc).cumsum(1).cumsum(2))


def test_moment_second_order_identity():
    # Mx(p,r,c) = r*H(p,r,c) - sum_{r'<r} H(p,r',c); My likewise along columns
    img = rand_img(np.random.default_rng(9), 1, 17, 23, 8)
    ih = oracle.ih(img, 4, 8).astype(np.int64)
    mx, my = oracle.moments(img, 4, 8)
    H, W = 17, 23
    ex = np.concatenate([np.zeros((4, 1, W), np.int64), ih.cumsum(1)[:, :-1]], axis=1)
    assert np.array_equal(mx, np.arange(H)[None, :, None] * ih - ex)
    ey = np.concatenate([np.zeros((4, H, 1), np.int64), ih.cumsum(2)[:, :, :-1]], axis=2)
    assert np.array_equal(my, np.arange(W)[None, None, :] * ih - ey)


def test_moments_constant_image_closed_form():
    H, W = 11, 8
    img = np.full((1, H, W), 3, np.uint8)
    mx, my = oracle.moments(img, 4, 8)
    assert mx[0, -1, -1] == W * H * (H - 1) // 2
    assert my[0, -1, -1] == H * W * (W - 1) // 2
    assert not mx[1:].any() and not my[1:].any()


# --------------------------------------------------------------------------- #
# Region query (Eq. 2.16)                                                     #
# --------------------------------------------------------------------------- #
def rand_rects(rng, H, W, n):
    r0 = rng.integers(0, H, n)
    c0 = rng.integers(0, W, n)
    r1 = np.array([rng.integers(a + 1, H + 1) for a in r0])
    c1 = np.array([rng.integers(a + 1, W + 1) for a in c0])
    return np.stack([r0, c0, r1, c1], 1).astype(np.int32)


def test_query_rect_vs_counting():
    rng = np.random.default_rng(10)
    C, H, W, bins = 2, 29, 41, 7
    img = rand_img(rng, C, H, W, 8)
    ih = oracle.ih(img, bins, 8)
    rects = rand_rects(rng, H, W, 300)
    q = oracle.query_rect(ih, rects)
    d = oracle.query_rect_direct(img, bins, 8, rects)
    assert np.array_equal(q, d)
    idx = oracle.plane_index(img, bins, 8)
    for i in range(0, 300, 17):
        r0, c0, r1, c1 = rects[i]
        ref = np.bincount(idx[:, r0:r1, c0:c1].ravel(), minlength=C * bins)
        assert np.array_equal(q[i], ref)


def test_query_rect_properties():
    rng = np.random.default_rng(11)
    C, H, W, bins = 1, 33, 40, 9
    img = rand_img(rng, C, H, W, 8)
    ih = oracle.ih(img, bins, 8)
    rects = rand_rects(rng, H, W, 200)
    q = oracle.query_rect(ih, rects).astype(np.int64)
    area = (rects[:, 2] - rects[:, 0]) * (rects[:, 3] - rects[:, 1])
    assert np.array_equal(q.sum(1), C * area)
    # split additivity, horizontally and vertically
    for i, (r0, c0, r1, c1) in enumerate(rects):
        rm, cm = (r0 + r1) // 2, (c0 + c1) // 2
        top, bot = oracle.query_rect(ih, [[r0, c0, rm, c1], [rm, c0, r1, c1]])
        left, right = oracle.query_rect(ih, [[r0, c0, r1, cm], [r0, cm, r1, c1]])
        assert np.array_equal(top + bot, q[i]) and np.array_equal(left + right, q[i])
        if i > 30:
            break
    full = oracle.query_rect(ih, [[0, 0, H, W]])[0]
    assert np.array_equal(full, ih[:, -1, -1])


def test_query_rect_edge_cases():
    img = rand_img(np.random.default_rng(12), 1, 6, 7, 8)
    ih = oracle.ih(img, 4, 8)
    out = oracle.query_rect(ih, [[2, 2, 2, 5], [0, 0, 7, 3], [-1, 0, 2, 2], [3, 4, 2, 5], [5, 6, 6, 7]])
    assert out[0].tolist() == [0] * 4         # empty
    assert out[1].tolist() == [-1] * 4        # r1 > H
    assert out[2].tolist() == [-1] * 4        # negative
    assert out[3].tolist() == [-1] * 4        # r0 > r1
    assert out[4].sum() == 1                  # single pixel


# --------------------------------------------------------------------------- #
# Spatially weighted histogram (Eq. 3.1, 3.3, 3.4; Sec. 3.1.3)                #
# --------------------------------------------------------------------------- #
def manhattan_total(h, w):
    """sum over the window of N(x,y); sum_x |2x - X| over h rows is 2*floor(h^2/4)."""
    return 2 * h * w * h * w - w * w * 2 * (h * h // 4) - h * h * 2 * (w * w // 4)


def swih_setup(seed, C=2, H=40, W=52, bins=6, n=150, lo=1, hi=30):
    rng = np.random.default_rng(seed)
    img = rand_img(rng, C, H, W, 8)
    ih = oracle.ih(img, bins, 8)
    mx, my = oracle.moments(img, bins, 8)
    h = rng.integers(lo, min(hi, H) + 1, n)
    w = rng.integers(lo, min(hi, W) + 1, n)
    r0 = np.array([rng.integers(0, H - a + 1) for a in h])
    c0 = np.array([rng.integers(0, W - a + 1) for a in w])
    rects = np.stack([r0, c0, r0 + h, c0 + w], 1).astype(np.int32)
    return img, ih, mx, my, rects, bins, C


def test_swih_numerator_exact_vs_bruteforce():
    # the thesis reports SWIH equal to brute force (MSE 0)
    img, ih, mx, my, rects, bins, C = swih_setup(13)
    num, val = oracle.weighted_swih(ih, mx, my, C, rects)
    assert np.array_equal(num, oracle.weighted_numerator(img, bins, 8, rects))
    bf = oracle.weighted_bruteforce(img, bins, 8, rects)
    np.testing.assert_allclose(val, bf, rtol=1e-6, atol=0)
    assert np.all((bf == 0) == (val == 0))


def test_swih_real_kernel_equals_integer_form():
    img, ih, mx, my, rects, bins, C = swih_setup(14)
    h = (rects[:, 2] - rects[:, 0]).astype(np.float64)
    w = (rects[:, 3] - rects[:, 1]).astype(np.float64)
    num = oracle.weighted_numerator(img, bins, 8, rects)
    bf = oracle.weighted_bruteforce(img, bins, 8, rects)
    np.testing.assert_allclose(bf, num / (2 * h * w)[:, None], rtol=1e-12, atol=1e-12)


def test_swih_l1_normalised():
    img, ih, mx, my, rects, bins, C = swih_setup(15)
    _, val = oracle.weighted_swih(ih, mx, my, C, rects, l1norm=True)
    bf = oracle.weighted_bruteforce(img, bins, 8, rects, l1norm=True)
    np.testing.assert_allclose(val, bf, rtol=1e-6, atol=1e-12)
    for ch in range(C):
        np.testing.assert_allclose(val[:, ch * bins:(ch + 1) * bins].sum(1), 1.0, rtol=1e-5)


def test_swih_channel_total_closed_form():
    img, ih, mx, my, rects, bins, C = swih_setup(16, lo=1, hi=40)
    num, val = oracle.weighted_swih(ih, mx, my, C, rects)
    h = rects[:, 2] - rects[:, 0]
    w = rects[:, 3] - rects[:, 1]
    for ch in range(C):
        tot = num[:, ch * bins:(ch + 1) * bins].sum(1)
        assert np.array_equal(tot, [manhattan_total(int(a), int(b)) for a, b in zip(h, w)])
    even = (h % 2 == 0) & (w % 2 == 0)
    np.testing.assert_allclose(val[even, :bins].sum(1), (h * w / 2.0)[even], rtol=1e-5)


def test_swih_single_pixel_is_plain():
    img, ih, mx, my, rects, bins, C = swih_setup(17, lo=1, hi=1)
    _, val = oracle.weighted_swih(ih, mx, my, C, rects)
    assert np.array_equal(val, oracle.query_rect(ih, rects).astype(np.float32))


def test_swih_translation_and_rotation_invariance():
    rng = np.random.default_rng(18)
    img = rand_img(rng, 1, 30, 30, 8)
    bins = 5
    win = np.array([[3, 4, 3 + 13, 4 + 10]], np.int32)
    base = oracle.weighted_numerator(img, bins, 8, win)
    # translate image and window together
    big = np.zeros((1, 45, 50), np.uint8)
    big[:, 7:37, 11:41] = img
    moved = oracle.weighted_numerator(big, bins, 8, win + np.array([7, 11, 7, 11], np.int32))
    assert np.array_equal(base, moved)
    # rotate the window's content by 180 degrees
    rot = img.copy()
    rot[:, 3:16, 4:14] = img[:, 3:16, 4:14][:, ::-1, ::-1]
    assert np.array_equal(base, oracle.weighted_numerator(rot, bins, 8, win))


def test_swih_golden(golden):
    g = golden("ih_3x4_2bins.txt")
    img = np.array(g["image"], dtype=np.uint8)[None]
    win = [[int(v) for v in g["window"][0]]]
    ih = oracle.ih(img, 2, 8)
    mx, my = oracle.moments(img, 2, 8)
    num, val = oracle.weighted_swih(ih, mx, my, 1, win)
    assert num[0].tolist() == [int(v) for v in g["weighted_numerator"][0]]
    np.testing.assert_allclose(oracle.weighted_bruteforce(img, 2, 8, win)[0],
                               [float(v) for v in g["weighted_hist"][0]], rtol=1e-15)
    np.testing.assert_allclose(val[0], [7 / 3, 8 / 3], rtol=1e-7)


def test_swih_invalid_and_empty():
    img, ih, mx, my, _, bins, C = swih_setup(19)
    num, val = oracle.weighted_swih(ih, mx, my, C, [[0, 0, 0, 5], [0, 0, 41, 5]])
    assert np.all(val[0] == 0) and np.all(np.isnan(val[1]))


# --------------------------------------------------------------------------- #
# Pyramid descriptor (Alg. 2, Sec. 2.4.4) and distances (Eq. 2.22-2.24)       #
# --------------------------------------------------------------------------- #
def test_pyramid_desc_vs_counting_and_levels():
    rng = np.random.default_rng(20)
    C, H, W, bins = 1, 50, 60, 8
    img = rand_img(rng, C, H, W, 8)
    ih = oracle.ih(img, bins, 8)
    wins = []
    for _ in range(60):
        h, w = int(rng.integers(1, 40)), int(rng.integers(1, 45))
        wins.append([int(rng.integers(0, H - h + 1)), int(rng.integers(0, W - w + 1)), h, w])
    d = oracle.pyramid_desc(ih, wins, 3)
    assert d.shape == (60, 21, bins)
    assert np.array_equal(d, oracle.pyramid_desc_direct(img, bins, 8, wins, 3))
    l0, l1, l2 = d[:, 0], d[:, 1:5], d[:, 5:21]
    assert np.array_equal(l1.sum(1), l0) and np.array_equal(l2.sum(1), l0)
    # each level-1 cell is the sum of its four level-2 children
    l2g = l2.reshape(60, 4, 4, bins)
    kids = l2g.reshape(60, 2, 2, 2, 2, bins).transpose(0, 1, 3, 2, 4, 5).reshape(60, 4, 4, bins).sum(2)
    assert np.array_equal(kids, l1)
    area = np.array([w[2] * w[3] for w in wins])
    assert np.array_equal(l0.sum(1), area)
    # brute force on one window: level-2 cell (1, 2) by slicing
    r, c, h, w = wins[0]
    rr = r + (1 * h) // 4, r + (2 * h) // 4
    cc = c + (2 * w) // 4, c + (3 * w) // 4
    idx = oracle.plane_index(img, bins, 8)[0]
    ref = np.bincount(idx[rr[0]:rr[1], cc[0]:cc[1]].ravel(), minlength=bins)
    assert np.array_equal(d[0, 5 + 1 * 4 + 2], ref)


def test_level_weights_eq_2_24_both_forms():
    for levels in (1, 2, 3, 4):
        L = levels - 1
        w = [oracle.level_weight(levels, l) for l in range(levels)]
        # second form of Eq. 2.24: 1/2^L for level 0, 1/2^(L-l+1) for l >= 1
        assert w[0] == 2.0 ** -L
        # first form: I^L + sum_{l<L} (I^l - I^{l+1}) / 2^(L-l); coefficient of I^l
        first = [0.0] * levels
        first[L] += 1.0
        for l in range(L):
            first[l] += 2.0 ** -(L - l)
            first[l + 1] -= 2.0 ** -(L - l)
        assert np.allclose(first, w)
    assert [oracle.level_weight(3, l) for l in range(3)] == [0.25, 0.25, 0.5]


def test_distances_hand_values():
    a = np.array([[1, 0]], np.int32)
    b = np.array([[0, 1]], np.int32)
    assert oracle.pyramid_distance(a, b, 1, "chi2") == 2.0      # 1/1 + 1/1
    assert oracle.pyramid_distance(a, b, 1, "l1") == 2.0
    assert oracle.pyramid_distance(a, b, 1, "pmk") == 0.0
    assert oracle.pyramid_distance(a, a, 1, "chi2") == 0.0
    z = np.zeros((1, 2), np.int32)
    assert oracle.pyramid_distance(z, z, 1, "chi2") == 0.0      # 0/0 := 0
    x = np.array([[4, 1, 0]], np.int32)
    y = np.array([[2, 3, 0]], np.int32)
    assert oracle.pyramid_distance(x, y, 1, "chi2") == pytest.approx(4 / 6 + 4 / 4)
    assert oracle.pyramid_distance(x, y, 1, "pmk") == 3.0


def test_distance_level_weighting():
    rng = np.random.default_rng(21)
    a = rng.integers(0, 20, (21, 5)).astype(np.int32)
    b = rng.integers(0, 20, (21, 5)).astype(np.int32)
    per = np.abs(a - b).sum(1).astype(np.float64)
    l1 = 0.25 * per[0] + 0.25 * per[1:5].sum() + 0.5 * per[5:].sum()
    assert oracle.pyramid_distance(a, b, 3, "l1") == l1
    mn = np.minimum(a, b).sum(1).astype(np.float64)
    assert oracle.pyramid_distance(a, b, 3, "pmk") == 0.25 * mn[0] + 0.25 * mn[1:5].sum() + 0.5 * mn[5:].sum()
    s = (a + b).astype(np.float64)
    t = np.where(s > 0, (a - b) ** 2 / np.where(s > 0, s, 1), 0.0).sum(1)
    assert oracle.pyramid_distance(a, b, 3, "chi2") == pytest.approx(0.25 * t[0] + 0.25 * t[1:5].sum() + 0.5 * t[5:].sum(), rel=1e-14)


def test_match_finds_template_origin():
    rng = np.random.default_rng(22)
    img = rand_img(rng, 1, 64, 70, 8)
    bins = 8
    tr, tc = 20, 25
    tmpl = oracle.pyramid_desc_direct(img, bins, 8, [[tr, tc, 12, 12]], 3)[0]
    origins = [(r, c) for r in range(10, 31) for c in range(15, 36)]
    for metric in ("chi2", "l1"):
        dist, best = oracle.match_direct(img, bins, 8, tmpl, 12, 12, 3, origins, metric)
        assert origins[best] == (tr, tc) and dist[best] == 0.0
        assert np.all(dist[np.arange(len(origins)) != best] > 0)
    sim, best = oracle.match_direct(img, bins, 8, tmpl, 12, 12, 3, origins, "pmk")
    assert origins[best] == (tr, tc) and sim[best] == 12 * 12


def test_match_borders_and_ties():
    img = np.zeros((1, 20, 20), np.uint8)
    tmpl = oracle.pyramid_desc_direct(img, 4, 8, [[0, 0, 4, 4]], 2)[0]
    origins = [(-1, 0), (17, 17), (3, 3), (5, 5)]
    dist, best = oracle.match_direct(img, 4, 8, tmpl, 4, 4, 2, origins, "chi2")
    assert np.isinf(dist[0]) and np.isinf(dist[1])
    assert best == 2                      # equal scores: the lowest index wins
    dist, best = oracle.match_direct(img, 4, 8, tmpl, 4, 4, 2, [(-1, 0)], "chi2")
    assert best == -1
