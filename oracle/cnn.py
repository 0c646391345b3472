"""FP64 NumPy oracle of the learned candidate-proposal network.

TEST INFRASTRUCTURE ONLY (imported by tests and the benchmark's CPU leg).

The thesis proposes no learned component; this network is the project's
reading of the "learned proposal" growth direction: a small convolutional
network that looks at a 7-channel crop centred on the previous target
position and scores every candidate offset of the exhaustive search, so that
only the best-scored candidates need exact pyramid scoring.

Network (shared definition with the GPU kernels, written independently):
  x   : 7 x 128 x 128 features (u8 / 255), rounded to BF16
  a1  = bf16(relu(conv(x,  W1, stride 2, pad 1) + b1))     32 x 64 x 64
  a2  = bf16(relu(conv(a1, W2, dilation 3, pad 3) + b2))   32 x 64 x 64
  a3  = bf16(relu(conv(a2, W3, dilation 9, pad 9) + b3))   32 x 64 x 64
  s   = sum_c wh[c] a3[c] + bh                             64 x 64
  L(dy,dx) = bilinear sample of s at (32 + dy/2, 32 + dx/2), dy,dx in [-32,32]
  loss = mean over the batch of -log softmax(L)[label]
Convolution weights are used as BF16 (rounded from FP32 masters); biases and
the head are FP32.  Backward mirrors the GPU's rounding points: the
pre-activation gradients dZ of each layer are rounded to BF16 before they
enter a product.  With ``exact=True`` nothing is rounded (FP64 throughout),
which is what the finite-difference pins check.
"""
from __future__ import annotations

import numpy as np

C_IN, C_MID, CROP, SMAP, RADIUS = 7, 32, 128, 64, 32
NOFF = 2 * RADIUS + 1           # 65 offsets per axis
# (cin, stride, dilation, pad); receptive field 3 + 2*3*2 + 2*9*2 = 51 input pixels
LAYERS = ((C_IN, 2, 1, 1), (C_MID, 1, 3, 3), (C_MID, 1, 9, 9))


# --------------------------------------------------------------- rounding --
def to_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def bf16(x):
    """Round to BF16 by round-to-nearest-even of the FP32 value, returned as float64."""
    f = to_f32(x)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


# ------------------------------------------------------------ convolution --
def conv(x, w, stride, dil, pad):
    """out[b,o,y,x] = sum_{i,kh,kw} w[o,i,kh,kw] * x[b,i, y*s + kh*d - p, x*s + kw*d - p] (zero outside)."""
    B, Ci, Hi, Wi = x.shape
    Co = w.shape[0]
    Ho = (Hi + 2 * pad - 2 * dil - 1) // stride + 1
    Wo = (Wi + 2 * pad - 2 * dil - 1) // stride + 1
    xp = np.zeros((B, Ci, Hi + 2 * pad, Wi + 2 * pad))
    xp[:, :, pad:pad + Hi, pad:pad + Wi] = x
    out = np.zeros((B, Co, Ho, Wo))
    for kh in range(3):
        for kw in range(3):
            patch = xp[:, :, kh * dil: kh * dil + stride * (Ho - 1) + 1: stride,
                       kw * dil: kw * dil + stride * (Wo - 1) + 1: stride]
            out += np.einsum("oi,biyx->boyx", w[:, :, kh, kw], patch)
    return out


def conv_transpose(dy, w, stride, dil, pad, in_shape):
    """Adjoint of conv: dx[b,i,y',x'] = sum over (o,kh,kw,y,x) mapping to (y',x') of w * dy."""
    B, Ci, Hi, Wi = in_shape
    Co, _, _, _ = w.shape
    Ho, Wo = dy.shape[2], dy.shape[3]
    dxp = np.zeros((B, Ci, Hi + 2 * pad, Wi + 2 * pad))
    for kh in range(3):
        for kw in range(3):
            dxp[:, :, kh * dil: kh * dil + stride * (Ho - 1) + 1: stride,
                kw * dil: kw * dil + stride * (Wo - 1) + 1: stride] += np.einsum("oi,boyx->biyx", w[:, :, kh, kw], dy)
    return dxp[:, :, pad:pad + Hi, pad:pad + Wi]


def conv_wgrad(x, dy, stride, dil, pad):
    """dW[o,i,kh,kw] = sum_{b,y,x} dy[b,o,y,x] * x[b,i, y*s + kh*d - p, x*s + kw*d - p]."""
    B, Ci, Hi, Wi = x.shape
    Co, Ho, Wo = dy.shape[1], dy.shape[2], dy.shape[3]
    xp = np.zeros((B, Ci, Hi + 2 * pad, Wi + 2 * pad))
    xp[:, :, pad:pad + Hi, pad:pad + Wi] = x
    dw = np.zeros((Co, Ci, 3, 3))
    for kh in range(3):
        for kw in range(3):
            patch = xp[:, :, kh * dil: kh * dil + stride * (Ho - 1) + 1: stride,
                       kw * dil: kw * dil + stride * (Wo - 1) + 1: stride]
            dw[:, :, kh, kw] = np.einsum("boyx,biyx->oi", dy, patch)
    return dw


# --------------------------------------------------------- offset sampling --
def sample_positions():
    """Score-map coordinates (u, v) of each of the 65 x 65 offsets."""
    d = np.arange(-RADIUS, RADIUS + 1)
    return SMAP // 2 + d / 2.0


def sample(s):
    """L[b, dy, dx] = bilinear(s[b], 32 + dy/2, 32 + dx/2)."""
    u = sample_positions()
    u0 = np.floor(u).astype(int)
    fu = u - u0
    u1 = np.minimum(u0 + 1, SMAP - 1)
    rows = s[:, u0, :] * (1 - fu)[None, :, None] + s[:, u1, :] * fu[None, :, None]
    return rows[:, :, u0] * (1 - fu)[None, None, :] + rows[:, :, u1] * fu[None, None, :]


def sample_transpose(dl):
    """Adjoint of sample: scatter dL back onto the score map."""
    B = dl.shape[0]
    u = sample_positions()
    u0 = np.floor(u).astype(int)
    fu = u - u0
    u1 = np.minimum(u0 + 1, SMAP - 1)
    ds_cols = np.zeros((B, NOFF, SMAP))
    np.add.at(ds_cols, (slice(None), slice(None), u0), dl * (1 - fu)[None, None, :])
    np.add.at(ds_cols, (slice(None), slice(None), u1), dl * fu[None, None, :])
    ds = np.zeros((B, SMAP, SMAP))
    np.add.at(ds, (slice(None), u0, slice(None)), ds_cols * (1 - fu)[None, :, None])
    np.add.at(ds, (slice(None), u1, slice(None)), ds_cols * fu[None, :, None])
    return ds


# ------------------------------------------------------------------ input --
def crop(feat, centers, side=CROP):
    """x[b,c,i,j] = bf16(feat[c, r - side/2 + i, q - side/2 + j] / 255) for the
    centre (r, q) of crop b; zero where the window leaves the frame."""
    C, H, W = feat.shape
    out = np.zeros((len(centers), C, side, side))
    for b, (r, q) in enumerate(centers):
        r0, q0 = int(r) - side // 2, int(q) - side // 2
        for i in range(side):
            if 0 <= r0 + i < H:
                for j in range(side):
                    if 0 <= q0 + j < W:
                        out[b, :, i, j] = feat[:, r0 + i, q0 + j] / 255.0
    return bf16(out)


# ------------------------------------------------------------ the network --
def init_params(seed):
    """He-normal FP32 initial parameters (the seeded initial state)."""
    rng = np.random.default_rng(seed)
    p = {}
    for i, (cin, _, _, _) in enumerate(LAYERS, 1):
        p["W%d" % i] = (rng.standard_normal((C_MID, cin, 3, 3)) * np.sqrt(2.0 / (cin * 9))).astype(np.float32)
        p["b%d" % i] = np.zeros(C_MID, np.float32)
    p["wh"] = (rng.standard_normal(C_MID) * np.sqrt(1.0 / C_MID)).astype(np.float32)
    p["bh"] = np.zeros(1, np.float32)
    return p


def forward(p, x, exact=False):
    """x: B x 7 x 128 x 128 in [0,1].  Returns (logits B x 65 x 65, cache)."""
    rnd = (lambda v: np.asarray(v, np.float64)) if exact else bf16
    a = rnd(x)
    cache = {"a0": a}
    for i, (cin, st, dl, pd) in enumerate(LAYERS, 1):
        w = rnd(p["W%d" % i])
        z = conv(a, w, st, dl, pd) + np.asarray(p["b%d" % i], np.float64)[None, :, None, None]
        a = rnd(np.maximum(z, 0.0))
        cache["a%d" % i] = a
    s = np.einsum("c,bcyx->byx", np.asarray(p["wh"], np.float64), a) + float(p["bh"][0])
    cache["s"] = s
    return sample(s), cache


def loss_and_grads(p, x, labels, exact=False):
    """Mean softmax cross-entropy over the 65*65 offsets and parameter gradients."""
    rnd = (lambda v: np.asarray(v, np.float64)) if exact else bf16
    logits, c = forward(p, x, exact)
    B = x.shape[0]
    flat = logits.reshape(B, -1)
    m = flat.max(1, keepdims=True)
    e = np.exp(flat - m)
    prob = e / e.sum(1, keepdims=True)
    loss = float(np.mean(-np.log(prob[np.arange(B), labels])))
    dl = prob.copy()
    dl[np.arange(B), labels] -= 1.0
    dl /= B
    ds = sample_transpose(dl.reshape(B, NOFF, NOFF))
    g = {"wh": np.einsum("byx,bcyx->c", ds, c["a3"]), "bh": np.array([ds.sum()])}
    da = np.einsum("byx,c->bcyx", ds, np.asarray(p["wh"], np.float64))
    for i in (3, 2, 1):
        cin, st, dl_, pd = LAYERS[i - 1]
        dz = rnd(da * (c["a%d" % i] > 0))
        g["W%d" % i] = conv_wgrad(c["a%d" % (i - 1)], dz, st, dl_, pd)
        g["b%d" % i] = dz.sum((0, 2, 3))
        if i > 1:
            da = conv_transpose(dz, rnd(p["W%d" % i]), st, dl_, pd, c["a%d" % (i - 1)].shape)
    return loss, g, logits


def sgd_step(p, g, v, lr, momentum=0.9, weight_decay=0.0):
    """v <- momentum*v + (g + wd*p);  p <- p - lr*v   (FP32 state)."""
    out_p, out_v = {}, {}
    for k in p:
        gk = np.asarray(g[k], np.float64) + weight_decay * np.asarray(p[k], np.float64)
        vk = momentum * np.asarray(v[k], np.float64) + gk
        out_v[k] = vk.astype(np.float32)
        out_p[k] = (np.asarray(p[k], np.float64) - lr * vk).astype(np.float32)
    return out_p, out_v


def topk(logits, k):
    """Indices of the k largest logits per sample, ties to the lower index."""
    flat = logits.reshape(logits.shape[0], -1)
    order = np.lexsort((np.arange(flat.shape[1])[None, :].repeat(flat.shape[0], 0), -flat), axis=1)
    return order[:, :k]
