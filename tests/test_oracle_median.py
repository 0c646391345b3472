"""Pins for the oracle's spatio-temporal median and joint integral histogram
(Alg. 4, Sec. 4.1.1).  The median is checked against numpy order statistics of
independently gathered samples, against the median read from the joint IH
through rectangle queries (the route Alg. 4 takes), and on special cases; the
joint IH against the sum of per-frame count IHs (pinned elsewhere) and
bincounts."""
import numpy as np
import pytest

import oracle


def video(seed, F, C, H, W, bits):
    rng = np.random.default_rng(seed)
    dt = np.uint8 if bits <= 8 else np.uint16
    return rng.integers(0, 1 << bits, size=(F, C, H, W)).astype(dt)


def window(r, c, H, W, wh, ww):
    return (max(0, r - (wh - 1) // 2), min(H, r + wh // 2 + 1), max(0, c - (ww - 1) // 2), min(W, c + ww // 2 + 1))


def numpy_median(frames, bins, bits, wh, ww):
    F, C, H, W = frames.shape
    b = (frames.astype(np.int64) * bins) >> bits
    out = np.empty((C, H, W), np.int64)
    for ch in range(C):
        for r in range(H):
            for c in range(W):
                r0, r1, c0, c1 = window(r, c, H, W, wh, ww)
                s = b[:, ch, r0:r1, c0:c1].ravel()
                out[ch, r, c] = np.partition(s, (s.size - 1) // 2)[(s.size - 1) // 2]
    return out


@pytest.mark.parametrize("F,C,H,W,bins,bits,wh,ww", [
    (1, 1, 6, 7, 8, 8, 1, 1), (3, 1, 9, 5, 16, 8, 3, 3), (5, 2, 8, 11, 4, 8, 3, 5),
    (4, 1, 7, 7, 64, 16, 2, 4), (17, 1, 6, 6, 256, 8, 5, 5), (2, 1, 5, 9, 3, 8, 9, 9)])
def test_median_matches_numpy_order_statistic(F, C, H, W, bins, bits, wh, ww):
    frames = video(F * 100 + H * W + wh, F, C, H, W, bits)
    assert np.array_equal(oracle.st_median(frames, bins, bits, wh, ww), numpy_median(frames, bins, bits, wh, ww))


@pytest.mark.parametrize("F,bins,wh,ww", [(3, 16, 3, 3), (6, 32, 5, 3), (17, 256, 3, 3)])
def test_median_from_joint_ih_queries(F, bins, wh, ww):
    """The Alg. 4 route: local histograms of the joint IH by four-corner
    queries, then the first bin whose running count reaches ceil(N/2)."""
    H, W = 13, 17
    frames = video(F + bins, F, 1, H, W, 8)
    J = oracle.jih(frames, bins, 8)
    rects = []
    for r in range(H):
        for c in range(W):
            r0, r1, c0, c1 = window(r, c, H, W, wh, ww)
            rects.append([r0, c0, r1, c1])
    rects = np.array(rects, np.int32)
    h = oracle.query_rect(J, rects).astype(np.int64)
    n = h.sum(1)
    area = (rects[:, 2] - rects[:, 0]) * (rects[:, 3] - rects[:, 1])
    assert np.array_equal(n, F * area)
    cum = np.cumsum(h, axis=1)
    med = np.argmax(cum >= ((n + 1) // 2)[:, None], axis=1).reshape(H, W)
    assert np.array_equal(oracle.st_median(frames, bins, 8, wh, ww)[0], med)


def test_joint_ih_is_sum_of_frame_ihs():
    frames = video(3, 5, 2, 19, 23, 8)
    ref = sum(oracle.ih(f, 16, 8).astype(np.int64) for f in frames)
    J = oracle.jih(frames, 16, 8)
    assert np.array_equal(J, ref)
    # last entry: bincount of every sample of the window
    for ch in range(2):
        b = (frames[:, ch].astype(np.int64) * 16) >> 8
        assert np.array_equal(J[ch * 16:(ch + 1) * 16, -1, -1], np.bincount(b.ravel(), minlength=16))


def test_joint_ih_sliding_update_identity():
    """Alg. 4's update: the window shifted by one frame equals the old joint IH
    plus the head frame's IH minus the tail frame's IH."""
    frames = video(4, 8, 1, 15, 21, 8)
    old = oracle.jih(frames[0:5], 32, 8).astype(np.int64)
    new = oracle.jih(frames[1:6], 32, 8).astype(np.int64)
    assert np.array_equal(new, old + oracle.ih(frames[5], 32, 8) - oracle.ih(frames[0], 32, 8))


def test_special_cases():
    frames = video(5, 1, 1, 9, 10, 8)
    # one frame, 1x1 window: the pixel's own bin
    assert np.array_equal(oracle.st_median(frames, 16, 8, 1, 1)[0], (frames[0, 0].astype(np.int64) * 16) >> 8)
    # constant video: that bin everywhere, whatever the window
    const = np.full((4, 1, 6, 8), 200, np.uint8)
    assert (oracle.st_median(const, 8, 8, 3, 5) == (200 * 8) >> 8).all()
    # three frames, 1x1 window: the middle bin of the three
    f3 = video(6, 3, 1, 7, 9, 8)
    b = (f3[:, 0].astype(np.int64) * 32) >> 8
    assert np.array_equal(oracle.st_median(f3, 32, 8, 1, 1)[0], np.sort(b, axis=0)[1])
    # the frame order does not matter
    f5 = video(7, 5, 1, 8, 8, 8)
    assert np.array_equal(oracle.st_median(f5, 16, 8, 3, 3), oracle.st_median(f5[::-1].copy(), 16, 8, 3, 3))


def test_hand_worked_example():
    """Two frames of a 2 x 2 image, 4 bins of 8-bit values (width 64), a 3 x 3
    window, which covers the whole image from every pixel: 8 samples with bins
    0,0,1,3 (frame 0) and 2,2,2,3 (frame 1), sorted 0,0,1,2,2,2,3,3, lower
    median at position 3 = bin 2."""
    frames = np.array([[[[10, 20], [70, 250]]], [[[130, 140], [150, 200]]]], np.uint8)
    assert (oracle.st_median(frames, 4, 8, 3, 3) == 2).all()
    # a 1 x 2 window spans columns c .. c+1 (clipped):
    #   (0,0): bins 0,0 | 2,2 -> 0,0,2,2 -> position 1 -> 0
    #   (0,1): bins 0 | 2     -> 0,2     -> position 0 -> 0
    #   (1,0): bins 1,3 | 2,3 -> 1,2,3,3 -> position 1 -> 2
    #   (1,1): bins 3 | 3     -> 3,3     -> position 0 -> 3
    assert oracle.st_median(frames, 4, 8, 1, 2)[0].tolist() == [[0, 0], [2, 3]]
