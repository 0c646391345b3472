"""Pins for the oracle's further spatial kernels (Fig. 3.1: quadratic, i.e.
squared Euclidean distance, and Gaussian), the second-moment integral
histograms, the O(1) quadratic-kernel route, and the wedding-cake
approximation (Eq. 3.2).  Checks use numpy cumulative sums, closed forms,
separability, numerical quadrature and direct per-pixel counting, each
independent of the oracle function it pins."""
import numpy as np
import pytest

import oracle


def rand_img(rng, C, H, W, bits=8):
    dt = np.uint8 if bits <= 8 else np.uint16
    return rng.integers(0, 1 << bits, size=(C, H, W)).astype(dt)


def rand_rects(rng, H, W, n, lo=1, hi=None):
    hi = hi or min(H, W)
    out = []
    for _ in range(n):
        h = int(rng.integers(lo, min(hi, H) + 1))
        w = int(rng.integers(lo, min(hi, W) + 1))
        r0 = int(rng.integers(0, H - h + 1))
        c0 = int(rng.integers(0, W - w + 1))
        out.append([r0, c0, r0 + h, c0 + w])
    return np.array(out, np.int32)


def test_second_moments_are_weighted_cumsums():
    rng = np.random.default_rng(1)
    img = rand_img(rng, 2, 17, 23)
    mxx, myy = oracle.moments2(img, 8, 8)
    b = (img.astype(np.int64) * 8) >> 8
    x = np.arange(17)[:, None] ** 2
    y = np.arange(23)[None, :] ** 2
    for ch in range(2):
        for k in range(8):
            one = (b[ch] == k).astype(np.int64)
            p = ch * 8 + k
            assert np.array_equal(mxx[p], np.cumsum(np.cumsum(one * x, 0), 1))
            assert np.array_equal(myy[p], np.cumsum(np.cumsum(one * y, 0), 1))


@pytest.mark.parametrize("l1norm", [False, True])
def test_quadratic_o1_route_equals_brute_force(l1norm):
    rng = np.random.default_rng(2)
    C, H, W, bins = 2, 40, 52, 6
    img = rand_img(rng, C, H, W)
    rects = rand_rects(rng, H, W, 60)
    ih = oracle.ih(img, bins, 8)
    mx, my = oracle.moments(img, bins, 8)
    mxx, myy = oracle.moments2(img, bins, 8)
    num, val = oracle.quadratic_swih(ih, mx, my, mxx, myy, C, rects, l1norm)
    assert np.array_equal(num, oracle.quadratic_numerator(img, bins, 8, rects))
    bf = oracle.kernel_bruteforce(img, bins, 8, rects, "quadratic", l1norm=l1norm)
    np.testing.assert_allclose(val, bf, rtol=2e-7, atol=1e-9)


def test_quadratic_total_weight_closed_form():
    """One bin: the numerator of the whole window is
    2h^3w^3 - w^3 h(h^2-1)/3 - h^3 w(w^2-1)/3."""
    img = np.zeros((1, 30, 40), np.uint8)
    rects = np.array([[0, 0, 30, 40], [3, 5, 4, 6], [2, 7, 9, 8], [10, 11, 27, 37]], np.int32)
    num = oracle.quadratic_numerator(img, 1, 8, rects)[:, 0]
    h = (rects[:, 2] - rects[:, 0]).astype(np.int64)
    w = (rects[:, 3] - rects[:, 1]).astype(np.int64)
    assert np.array_equal(num, 2 * h**3 * w**3 - w**3 * h * (h * h - 1) // 3 - h**3 * w * (w * w - 1) // 3)
    # the kernel is 1 at the centre pixel of an odd window and 0 beyond the corners
    bf = oracle.kernel_bruteforce(img, 1, 8, np.array([[0, 0, 1, 1]], np.int32), "quadratic")
    assert bf[0, 0] == 1.0


def test_gaussian_is_separable():
    img = np.zeros((1, 25, 31), np.uint8)
    rects = np.array([[0, 0, 25, 31], [4, 6, 15, 29]], np.int32)
    for s in (0.3, 0.5, 1.0):
        bf = oracle.kernel_bruteforce(img, 1, 8, rects, "gaussian", sigma=s)[:, 0]
        for i, (r0, c0, r1, c1) in enumerate(rects):
            h, w = r1 - r0, c1 - c0
            u = (np.arange(r0, r1) - (r0 + r1 - 1) / 2) / (h / 2)
            v = (np.arange(c0, c1) - (c0 + c1 - 1) / 2) / (w / 2)
            ref = np.exp(-u**2 / (2 * s * s)).sum() * np.exp(-v**2 / (2 * s * s)).sum()
            assert abs(bf[i] - ref) < 1e-9 * ref


def test_manhattan_kernel_matches_weighted_bruteforce():
    rng = np.random.default_rng(3)
    img = rand_img(rng, 2, 30, 30)
    rects = rand_rects(rng, 30, 30, 20)
    for l1 in (False, True):
        np.testing.assert_allclose(oracle.kernel_bruteforce(img, 5, 8, rects, "manhattan", l1norm=l1),
                                   oracle.weighted_bruteforce(img, 5, 8, rects, l1), rtol=1e-12)


@pytest.mark.parametrize("kernel,sigma", [("manhattan", 0.5), ("quadratic", 0.5), ("gaussian", 0.4),
                                          ("gaussian", 1.5)])
@pytest.mark.parametrize("h,w,L", [(60, 60, 5), (37, 81, 4), (9, 14, 3)])
def test_ring_weights_are_annulus_means(kernel, sigma, h, w, L):
    """Midpoint-rule means of the kernel over each ring, the ring being the
    normalised rectangle of layer j minus that of layer j-1 (layer margins
    floor((L-j) h / 2L) rows and floor((L-j) w / 2L) columns)."""
    wts = oracle.ring_weights(h, w, L, kernel, sigma)
    g = (np.arange(2000) + 0.5) / 1000 - 1.0
    u, v = np.meshgrid(g, g, indexing="ij")
    if kernel == "manhattan":
        K = 1 - 0.5 * (np.abs(u) + np.abs(v))
    elif kernel == "quadratic":
        K = 1 - 0.5 * (u * u + v * v)
    else:
        K = np.exp(-(u * u + v * v) / (2 * sigma * sigma))
    inside_prev = np.zeros_like(u, bool)
    for j in range(1, L + 1):
        a = 1 - 2 * (((L - j) * h) // (2 * L)) / h
        b = 1 - 2 * (((L - j) * w) // (2 * L)) / w
        inside = (np.abs(u) <= a) & (np.abs(v) <= b)
        ring = inside & ~inside_prev
        if ring.sum() > 2000:
            assert abs(wts[j - 1] - K[ring].mean()) < 3e-3, j
        inside_prev = inside


def test_wedding_ih_route_equals_direct_counting():
    rng = np.random.default_rng(4)
    C, H, W, bins = 2, 45, 50, 7
    img = rand_img(rng, C, H, W)
    rects = rand_rects(rng, H, W, 50)
    ih = oracle.ih(img, bins, 8)
    for L in (1, 2, 3, 5, 8):
        for kernel in ("manhattan", "quadratic", "gaussian"):
            a = oracle.wedding(ih, rects, L, kernel, 0.5)
            b = oracle.wedding_direct(img, bins, 8, rects, L, kernel, 0.5)
            np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


def test_wedding_special_cases():
    rng = np.random.default_rng(5)
    H, W, bins = 40, 40, 4
    img = rand_img(rng, 1, H, W)
    rects = rand_rects(rng, H, W, 30)
    ih = oracle.ih(img, bins, 8)
    plain = oracle.query_rect(ih, rects).astype(np.float64)
    # one layer: the annulus is the whole square, weight = the kernel's mean
    np.testing.assert_allclose(oracle.wedding(ih, rects, 1, "manhattan"), 0.5 * plain, rtol=1e-12)
    np.testing.assert_allclose(oracle.wedding(ih, rects, 1, "quadratic"), plain * 2 / 3, rtol=1e-12)
    # a very wide Gaussian weighs every ring ~1: the plain histogram
    np.testing.assert_allclose(oracle.wedding(ih, rects, 4, "gaussian", 1e4), plain, rtol=1e-7)


def test_wedding_error_shrinks_with_layers():
    """Eq. 3.2 gets closer to the exact kernel histogram as layers are added,
    down to a floor: none of these kernels is constant on a square ring."""
    rng = np.random.default_rng(6)
    H, W, bins = 90, 90, 8
    img = rand_img(rng, 1, H, W)
    rects = rand_rects(rng, H, W, 40, lo=40, hi=90)
    ih = oracle.ih(img, bins, 8)
    for kernel in ("manhattan", "quadratic", "gaussian"):
        exact = oracle.kernel_bruteforce(img, bins, 8, rects, kernel, sigma=0.5)
        err = [np.abs(oracle.wedding(ih, rects, L, kernel, 0.5) - exact).mean() / np.abs(exact).mean()
               for L in (1, 3, 16)]
        assert err[0] > err[1] > err[2] > 1e-3, (kernel, err)
        # the total weight of a one-bin window is right at every layer count
        one = np.zeros((1, H, W), np.uint8)
        ex1 = oracle.kernel_bruteforce(one, 1, 8, rects, kernel, sigma=0.5)
        for L in (1, 3, 16):
            np.testing.assert_allclose(oracle.wedding(oracle.ih(one, 1, 8), rects, L, kernel, 0.5), ex1, rtol=2e-3)
