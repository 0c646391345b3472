"""Pins for the FP64 proposal-network oracle: explicit loop nests, adjoint
identities, finite differences of the unrounded network, BF16 rounding."""
import numpy as np
import pytest

from oracle import cnn


def loop_conv(x, w, stride, dil, pad):
    B, Ci, Hi, Wi = x.shape
    Co = w.shape[0]
    Ho = (Hi + 2 * pad - 2 * dil - 1) // stride + 1
    Wo = (Wi + 2 * pad - 2 * dil - 1) // stride + 1
    out = np.zeros((B, Co, Ho, Wo))
    for b in range(B):
        for o in range(Co):
            for y in range(Ho):
                for xx in range(Wo):
                    acc = 0.0
                    for i in range(Ci):
                        for kh in range(3):
                            for kw in range(3):
                                r, c = y * stride + kh * dil - pad, xx * stride + kw * dil - pad
                                if 0 <= r < Hi and 0 <= c < Wi:
                                    acc += w[o, i, kh, kw] * x[b, i, r, c]
                    out[b, o, y, xx] = acc
    return out


@pytest.mark.parametrize("stride,dil,pad", [(1, 1, 1), (2, 1, 1), (1, 2, 2), (1, 3, 3), (1, 9, 9), (2, 2, 1)])
def test_conv_equals_loop_nest(stride, dil, pad):
    rng = np.random.default_rng(stride * 10 + dil)
    x = rng.standard_normal((2, 3, 11, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    np.testing.assert_allclose(cnn.conv(x, w, stride, dil, pad), loop_conv(x, w, stride, dil, pad), rtol=1e-12,
                               atol=1e-12)


@pytest.mark.parametrize("stride,dil,pad", [(1, 3, 3), (2, 1, 1), (1, 9, 9)])
def test_conv_adjoint_identities(stride, dil, pad):
    rng = np.random.default_rng(7 + dil)
    x = rng.standard_normal((2, 3, 16, 13))
    w = rng.standard_normal((5, 3, 3, 3))
    y = rng.standard_normal(cnn.conv(x, w, stride, dil, pad).shape)
    lhs = np.sum(cnn.conv(x, w, stride, dil, pad) * y)
    assert np.isclose(lhs, np.sum(x * cnn.conv_transpose(y, w, stride, dil, pad, x.shape)), rtol=1e-12)
    assert np.isclose(lhs, np.sum(w * cnn.conv_wgrad(x, y, stride, dil, pad)), rtol=1e-12)


def test_sampling_bilinear_and_adjoint():
    rng = np.random.default_rng(3)
    s = rng.standard_normal((2, cnn.SMAP, cnn.SMAP))
    L = cnn.sample(s)
    assert L.shape == (2, cnn.NOFF, cnn.NOFF)
    # even offsets land on grid points; odd offsets are midpoints
    assert L[0, 32, 32] == s[0, 32, 32]
    assert L[1, 34, 30] == s[1, 33, 31]
    assert np.isclose(L[0, 33, 32], 0.5 * (s[0, 32, 32] + s[0, 33, 32]))
    assert np.isclose(L[0, 33, 35], 0.25 * (s[0, 32, 33] + s[0, 33, 33] + s[0, 32, 34] + s[0, 33, 34]))
    dl = rng.standard_normal(L.shape)
    assert np.isclose(np.sum(L * dl), np.sum(s * cnn.sample_transpose(dl)), rtol=1e-12)


def test_bf16_rounding():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 3.0e-3, 0.0, 1 + 2 ** -7])
    r = cnn.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0                    # tie to even
    assert r[2] == 1 + 2 ** -6                            # tie to even (up)
    assert r[3] == -2.5 and r[5] == 0.0 and r[6] == 1 + 2 ** -7
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2 ** -8
    x = np.random.default_rng(0).standard_normal(1000)
    assert np.all(np.abs(cnn.bf16(x) - x) <= np.abs(x) * 2 ** -8)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(11)
    p = cnn.init_params(5)
    p = {k: (v + 0.05 * rng.standard_normal(v.shape)).astype(np.float32) for k, v in p.items()}
    x = rng.random((1, cnn.C_IN, cnn.CROP, cnn.CROP))
    labels = np.array([int(rng.integers(0, cnn.NOFF * cnn.NOFF))])
    _, g, _ = cnn.loss_and_grads(p, x, labels, exact=True)
    eps = 1e-6   # small enough that no ReLU kink is crossed for these seeds
    for name, idxs in (("W1", [(3, 2, 1, 1), (17, 6, 0, 2)]), ("W2", [(0, 5, 2, 2)]), ("W3", [(31, 31, 1, 0)]),
                       ("b1", [(4,)]), ("b3", [(9,)]), ("wh", [(2,), (30,)]), ("bh", [(0,)])):
        for ix in idxs:
            pp = {k: v.astype(np.float64) for k, v in p.items()}
            pm = {k: v.astype(np.float64) for k, v in p.items()}
            pp[name][ix] += eps
            pm[name][ix] -= eps
            lp, _, _ = cnn.loss_and_grads(pp, x, labels, exact=True)
            lm, _, _ = cnn.loss_and_grads(pm, x, labels, exact=True)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[name][ix]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, ix, fd, g[name][ix])


def test_loss_gradient_of_logits_sums_to_zero_and_topk_ties():
    p = cnn.init_params(1)
    x = np.random.default_rng(2).random((2, cnn.C_IN, cnn.CROP, cnn.CROP))
    loss, g, logits = cnn.loss_and_grads(p, x, np.array([0, 4224]))
    assert np.isfinite(loss) and loss > 0
    assert abs(g["bh"][0]) < 1e-12                        # sum of (softmax - onehot) is zero
    L = np.zeros((1, 5))
    L[0, [1, 3]] = 2.0
    assert cnn.topk(L, 3).tolist() == [[1, 3, 0]]


def test_sgd_step():
    p = {"a": np.array([1.0, -2.0], np.float32)}
    g = {"a": np.array([0.5, 0.5])}
    v = {"a": np.array([1.0, 0.0], np.float32)}
    p2, v2 = cnn.sgd_step(p, g, v, lr=0.1, momentum=0.9, weight_decay=0.0)
    assert np.allclose(v2["a"], [1.4, 0.5]) and np.allclose(p2["a"], [0.86, -2.05])


def test_crop_window_and_border():
    feat = np.arange(3 * 5 * 6, dtype=np.uint8).reshape(3, 5, 6) * 2
    x = cnn.crop(feat, [(2, 3), (0, 0)], side=4)
    # centre (2,3): rows 0..3, columns 1..4 of the frame
    np.testing.assert_array_equal(x[0], cnn.bf16(feat[:, 0:4, 1:5] / 255.0))
    # centre (0,0): rows -2..1, columns -2..1; only the lower-right 2x2 is inside
    assert np.all(x[1, :, :2, :] == 0) and np.all(x[1, :, :, :2] == 0)
    np.testing.assert_array_equal(x[1, :, 2:, 2:], cnn.bf16(feat[:, 0:2, 0:2] / 255.0))
    full = cnn.crop(np.full((1, 2, 2), 255, np.uint8), [(1, 1)], side=2)
    assert np.all(full == 1.0)
