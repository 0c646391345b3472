"""Pins for the oracle's weighted integral histogram (Alg. 2 step 4: the
gradient-magnitude weighted integral histogram of gradient orientation over
edge pixels).  Each check ties it to something other than its own recurrence:
the defining double sum, the count histogram (itself pinned to brute force),
a layer-cake decomposition of the weights into count histograms, weighted
bincounts and cumulative sums taken by numpy."""
import numpy as np
import pytest

import oracle


def rand_case(rng, C, H, W, bits, wmax=255, mask_p=0.5):
    dt = np.uint8 if bits <= 8 else np.uint16
    img = rng.integers(0, 1 << bits, size=(C, H, W)).astype(dt)
    wt = rng.integers(0, wmax + 1, size=(C, H, W)).astype(np.uint8)
    mask = (rng.random((C, H, W)) < mask_p).astype(np.uint8) * rng.integers(1, 256, size=(C, H, W)).astype(np.uint8)
    return img, wt, mask


def eff_weight(wt, mask):
    return wt.astype(np.int64) * (mask != 0) if mask is not None else wt.astype(np.int64)


@pytest.mark.parametrize("C,H,W,bins,bits", [(1, 5, 7, 3, 8), (2, 6, 4, 4, 8), (1, 4, 9, 5, 10), (3, 3, 3, 2, 16)])
@pytest.mark.parametrize("use_mask", [False, True])
def test_recurrence_equals_double_sum(C, H, W, bins, bits, use_mask):
    rng = np.random.default_rng(H * 100 + W * 10 + bins + use_mask)
    img, wt, mask = rand_case(rng, C, H, W, bits)
    m = mask if use_mask else None
    a = oracle.ih_weighted(img, bins, bits, wt, m)
    b = oracle.ih_weighted(img, bins, bits, wt, m, brute=True)
    assert np.array_equal(a, b)


def test_unit_weights_give_count_histogram():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, size=(2, 37, 53)).astype(np.uint8)
    ones = np.ones_like(img)
    assert np.array_equal(oracle.ih_weighted(img, 16, 8, ones), oracle.ih(img, 16, 8))
    # a mask of all non-zero bytes changes nothing
    full = np.full_like(img, 7)
    assert np.array_equal(oracle.ih_weighted(img, 16, 8, ones, full), oracle.ih(img, 16, 8))


def test_layer_cake_of_count_histograms():
    """A weight w is the sum over t = 1..w of 1, so the weighted histogram is
    the sum over t of count histograms of the pixels whose weight is >= t.
    Each of those is a count histogram of an image in which the other pixels
    are moved to extra bins beyond the real ones (value + 256 with one more
    value bit and twice the bins keeps every real bin where it was)."""
    rng = np.random.default_rng(2)
    C, H, W, bins = 1, 23, 31, 8
    img, wt, mask = rand_case(rng, C, H, W, 8, wmax=5)
    w = eff_weight(wt, mask)
    total = np.zeros((C * bins, H, W), np.int64)
    for t in range(1, int(w.max()) + 1):
        moved = img.astype(np.uint16) + np.where(w >= t, 0, 256).astype(np.uint16)
        ih_t = oracle.ih(moved, 2 * bins, 9)          # 2*bins planes, real ones first
        total += ih_t[:bins]
    assert np.array_equal(oracle.ih_weighted(img, bins, 8, wt, mask), total)


@pytest.mark.parametrize("bins,bits", [(16, 8), (7, 8), (64, 16)])
def test_last_entry_is_weighted_bincount(bins, bits):
    rng = np.random.default_rng(bins)
    C, H, W = 2, 41, 29
    img, wt, mask = rand_case(rng, C, H, W, bits)
    G = oracle.ih_weighted(img, bins, bits, wt, mask)
    w = eff_weight(wt, mask)
    for ch in range(C):
        # equal-width bins of the value range, assigned with numpy's digitize
        edges = np.arange(1, bins) * (1 << bits) / bins
        b = np.digitize(img[ch].astype(np.float64).ravel(), edges)
        ref = np.bincount(b, weights=w[ch].ravel(), minlength=bins).astype(np.int64)
        assert np.array_equal(G[ch * bins:(ch + 1) * bins, -1, -1], ref)


def test_sum_over_bins_is_cumulative_weight():
    rng = np.random.default_rng(3)
    C, H, W, bins = 3, 19, 44, 5
    img, wt, mask = rand_case(rng, C, H, W, 8)
    G = oracle.ih_weighted(img, bins, 8, wt, mask).astype(np.int64)
    w = eff_weight(wt, mask)
    for ch in range(C):
        s = G[ch * bins:(ch + 1) * bins].sum(axis=0)
        assert np.array_equal(s, np.cumsum(np.cumsum(w[ch], axis=0), axis=1))


def test_rect_queries_give_weighted_region_histograms():
    rng = np.random.default_rng(4)
    H, W, bins = 30, 40, 6
    img, wt, mask = rand_case(rng, 1, H, W, 8)
    G = oracle.ih_weighted(img, bins, 8, wt, mask)
    rects = np.array([[0, 0, H, W], [3, 5, 17, 29], [10, 10, 11, 11], [0, 7, 30, 8], [5, 5, 5, 9]], np.int32)
    q = oracle.query_rect(G, rects)
    w = eff_weight(wt, mask)[0]
    b = (img[0].astype(np.int64) * bins) >> 8
    for i, (r0, c0, r1, c1) in enumerate(rects):
        ref = np.bincount(b[r0:r1, c0:c1].ravel(), weights=w[r0:r1, c0:c1].ravel(), minlength=bins)
        assert np.array_equal(q[i], ref.astype(np.int64))


def test_zero_mask_and_zero_weight():
    rng = np.random.default_rng(5)
    img, wt, _ = rand_case(rng, 1, 9, 11, 8)
    assert not oracle.ih_weighted(img, 4, 8, wt, np.zeros_like(wt)).any()
    assert not oracle.ih_weighted(img, 4, 8, np.zeros_like(wt)).any()


def test_hand_worked_example():
    """2 x 3 image, 2 bins of 8-bit values (bin 0: 0..127, bin 1: 128..255)."""
    img = np.array([[[10, 200, 130], [127, 128, 0]]], np.uint8)
    wt = np.array([[[3, 4, 5], [6, 7, 8]]], np.uint8)
    mask = np.array([[[1, 1, 0], [1, 0, 1]]], np.uint8)
    G = oracle.ih_weighted(img, 2, 8, wt, mask)
    # bin 0 pixels with mask set: (0,0) w3, (1,0) w6, (1,2) w8
    # bin 1 pixels with mask set: (0,1) w4   ((0,2) and (1,1) are masked out)
    assert G[0].tolist() == [[3, 3, 3], [9, 9, 17]]
    assert G[1].tolist() == [[0, 4, 4], [0, 4, 4]]


def test_overflow_is_reported():
    H, W = 3000, 3000                      # 9 M pixels of weight 255 exceed 2^31 - 1
    img = np.zeros((1, H, W), np.uint8)
    wt = np.full((1, H, W), 255, np.uint8)
    with pytest.raises(RuntimeError):
        oracle.ih_weighted(img, 1, 8, wt)


def test_shape_checks():
    img = np.zeros((1, 4, 5), np.uint8)
    with pytest.raises(ValueError):
        oracle.ih_weighted(img, 2, 8, np.zeros((1, 5, 4), np.uint8))
    with pytest.raises(ValueError):
        oracle.ih_weighted(img, 2, 8, np.zeros((1, 4, 5), np.uint8), np.zeros((4, 5), np.uint8))
