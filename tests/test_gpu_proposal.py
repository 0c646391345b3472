"""Parity of the learned-proposal kernels (ih_lp_*) with the FP64 oracle.

Each kernel is checked on the same BF16 inputs as the oracle.  Bounds:
  * a sum of n FP32 products, accumulated in any order, is within
    n * 2^-24 * sum|terms| of the exact sum (gamma_n); the FP64 oracle is exact
    to far below that;
  * a BF16 result is rounded from that FP32 value, so it must lie between the
    BF16 roundings of (exact - bound) and (exact + bound) (rounding is monotonic);
  * gradients additionally meet the 1e-3 norm-relative bar.
"""
import numpy as np
import pytest
import torch

from oracle import cnn
from synth import smooth

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_01656_amd import proposal
    proposal.lib()
    return proposal


def bf(a, dev="cuda"):
    """Host FP64 values that are already BF16-exact -> device bf16 tensor."""
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev).to(torch.bfloat16)


def host(t):
    return t.float().cpu().numpy().astype(np.float64)


def bracket(gpu, exact, bound, relu=False):
    """gpu (BF16) equals a BF16 rounding of some value within bound of exact."""
    f = (lambda v: np.maximum(v, 0.0)) if relu else (lambda v: v)
    lo, hi = cnn.bf16(f(exact - bound)), cnn.bf16(f(exact + bound))
    ok = (gpu >= lo) & (gpu <= hi)
    assert ok.all(), "%d of %d outside; first at %s: gpu %r exact %r bound %r" % (
        (~ok).sum(), ok.size, np.argwhere(~ok)[0], gpu[~ok][0], exact[~ok][0], bound[~ok][0])
    return np.mean(gpu == cnn.bf16(f(exact)))


def rand_act(rng, shape, frac_zero=0.4):
    v = rng.standard_normal(shape) * 0.7
    v[rng.random(shape) < frac_zero] = 0.0
    return cnn.bf16(np.abs(v))


def pack_w(w):
    """[32][Cin][3][3] -> [32][9][Cpad] tap-major, channels zero-padded to 8."""
    co, ci = w.shape[:2]
    cpad = (ci + 7) // 8 * 8
    out = np.zeros((co, 9, cpad))
    out[:, :, :ci] = w.reshape(co, ci, 9).transpose(0, 2, 1)
    return out.reshape(co, 9 * cpad)


def flip_t(w):
    """Input-gradient operand: wt[ci][co][kh][kw] = w[co][ci][2-kh][2-kw]."""
    return np.ascontiguousarray(w[:, :, ::-1, ::-1].transpose(1, 0, 2, 3))


CONV_CASES = [  # B, Cin, Hin, Win, stride, dil, pad
    (2, 7, 128, 128, 2, 1, 1),     # layer 1 of the network
    (2, 32, 64, 64, 1, 3, 3),      # layer 2
    (1, 32, 64, 64, 1, 9, 9),      # layer 3
    (1, 32, 40, 24, 1, 2, 2),      # another dilation
    (1, 5, 37, 23, 2, 1, 1),       # ragged: 228 output pixels, K = 45
    (3, 3, 9, 11, 1, 2, 2),        # tiny, K = 27
]


@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_forward(P, case):
    B, Cin, Hin, Win, st, d, pd = case
    rng = np.random.default_rng(sum(case))
    x = rand_act(rng, (B, Cin, Hin, Win))
    w = cnn.bf16(rng.standard_normal((32, Cin, 3, 3)) * np.sqrt(2.0 / (Cin * 9)))
    b = cnn.to_f32(rng.standard_normal(32) * 0.1).astype(np.float64)
    z = cnn.conv(x, w, st, d, pd) + b[None, :, None, None]
    mag = cnn.conv(np.abs(x), np.abs(w), st, d, pd) + np.abs(b)[None, :, None, None]
    out = torch.empty(z.shape, dtype=torch.bfloat16, device="cuda")
    P.lp_conv(bf(x), bf(pack_w(w)), torch.from_numpy(b.astype(np.float32)).cuda(), st, d, pd, out)
    torch.cuda.synchronize()
    exact_frac = bracket(host(out), z, (Cin * 9 + 2) * U * mag, relu=True)
    assert exact_frac > 0.99


@pytest.mark.parametrize("case", [(2, 32, 64, 64, 1, 3, 3), (1, 32, 64, 64, 1, 9, 9), (2, 32, 19, 13, 1, 2, 2)])
def test_conv_input_gradient(P, case):
    B, Cin, H, W, st, d, pd = case
    rng = np.random.default_rng(100 + sum(case))
    a_prev = rand_act(rng, (B, Cin, H, W))                       # mask: input activation of the layer
    dz = cnn.bf16(rng.standard_normal((B, 32, H, W)) * 1e-3)
    w = cnn.bf16(rng.standard_normal((32, Cin, 3, 3)) * 0.08)
    da = cnn.conv_transpose(dz, w, st, d, pd, a_prev.shape)
    mag = cnn.conv_transpose(np.abs(dz), np.abs(w), st, d, pd, a_prev.shape)
    keep = a_prev > 0
    out = torch.empty(a_prev.shape, dtype=torch.bfloat16, device="cuda")
    P.lp_conv(bf(dz), bf(pack_w(flip_t(w))), None, 1, d, pd, out, mask=bf(a_prev))
    torch.cuda.synchronize()
    g = host(out)
    assert np.all(g[~keep] == 0)
    exact_frac = bracket(g[keep], da[keep], (32 * 9 + 1) * U * mag[keep])
    assert exact_frac > 0.99


@pytest.mark.parametrize("case,chunk", [((2, 7, 128, 128, 2, 1, 1), 1024), ((2, 32, 64, 64, 1, 3, 3), 1024),
                                        ((1, 32, 64, 64, 1, 9, 9), 512), ((1, 5, 37, 23, 2, 1, 1), 64),
                                        ((3, 3, 9, 11, 1, 2, 2), 8)])
def test_conv_weight_gradient(P, case, chunk):
    B, Cin, Hin, Win, st, d, pd = case
    rng = np.random.default_rng(200 + sum(case))
    x = rand_act(rng, (B, Cin, Hin, Win))
    Ho = (Hin + 2 * pd - 2 * d - 1) // st + 1
    Wo = (Win + 2 * pd - 2 * d - 1) // st + 1
    dz = cnn.bf16(rng.standard_normal((B, 32, Ho, Wo)) * 1e-3)
    dw_ref = cnn.conv_wgrad(x, dz, st, d, pd)
    mag = cnn.conv_wgrad(np.abs(x), np.abs(dz), st, d, pd)
    db_ref, db_mag = dz.sum((0, 2, 3)), np.abs(dz).sum((0, 2, 3))
    dw = torch.empty(32 * Cin * 9, dtype=torch.float32, device="cuda")
    db = torch.empty(32, dtype=torch.float32, device="cuda")
    P.lp_wgrad(bf(x), bf(dz), st, d, pd, dw, db, chunk=chunk)
    torch.cuda.synchronize()
    n = B * Ho * Wo
    g, gb = host(dw).reshape(dw_ref.shape), host(db)
    assert np.all(np.abs(g - dw_ref) <= n * U * mag + 1e-30)
    assert np.all(np.abs(gb - db_ref) <= n * U * db_mag + 1e-30)
    assert np.linalg.norm(g - dw_ref) <= 1e-3 * np.linalg.norm(dw_ref)


def test_wgrad_is_deterministic(P):
    rng = np.random.default_rng(5)
    x = bf(rand_act(rng, (4, 32, 64, 64)))
    dz = bf(cnn.bf16(rng.standard_normal((4, 32, 64, 64)) * 1e-3))
    outs = []
    for _ in range(3):
        dw = torch.empty(32 * 288, dtype=torch.float32, device="cuda")
        db = torch.empty(32, dtype=torch.float32, device="cuda")
        P.lp_wgrad(x, dz, 1, 3, 3, dw, db)
        outs.append((dw.cpu(), db.cpu()))
    for dw, db in outs[1:]:
        assert torch.equal(dw, outs[0][0]) and torch.equal(db, outs[0][1])


def test_head_logits(P):
    rng = np.random.default_rng(7)
    a3 = rand_act(rng, (3, 32, 64, 64))
    wh = cnn.to_f32(rng.standard_normal(32) * 0.2).astype(np.float64)
    bh = cnn.to_f32([0.3]).astype(np.float64)
    s = np.einsum("c,bcyx->byx", wh, a3) + bh[0]
    ref = cnn.sample(s)
    mag = cnn.sample(np.einsum("c,bcyx->byx", np.abs(wh), a3) + abs(bh[0]))
    logits = torch.empty((3, 65, 65), dtype=torch.float32, device="cuda")
    P.lp_head(bf(a3), torch.tensor(wh, dtype=torch.float32, device="cuda"),
              torch.tensor(bh, dtype=torch.float32, device="cuda"), logits)
    torch.cuda.synchronize()
    assert np.all(np.abs(host(logits) - ref) <= 40 * U * mag)


def test_softmax_ce(P):
    rng = np.random.default_rng(8)
    B = 5
    L = cnn.to_f32(rng.standard_normal((B, 4225)) * 3).astype(np.float64)
    labels = rng.integers(0, 4225, B)
    labels[0], labels[1] = 0, 4224
    m = L.max(1, keepdims=True)
    lse = np.log(np.exp(L - m).sum(1, keepdims=True)) + m
    loss_ref = (lse[:, 0] - L[np.arange(B), labels])
    prob = np.exp(L - lse)
    d_ref = prob.copy()
    d_ref[np.arange(B), labels] -= 1
    d_ref /= B
    Lt = torch.tensor(L, dtype=torch.float32, device="cuda")
    loss = torch.empty(B, dtype=torch.float32, device="cuda")
    dl = torch.empty_like(Lt)
    P.lp_softmax_ce(Lt, torch.tensor(labels, dtype=torch.int32, device="cuda"), loss, dl)
    torch.cuda.synchronize()
    np.testing.assert_allclose(host(loss), loss_ref, rtol=1e-5, atol=1e-5)
    assert np.all(np.abs(host(dl) - d_ref) <= 1e-5 * (prob + 1.0 * (d_ref < 0)) / B + 1e-12)
    # the per-sample gradient sums to zero
    assert np.all(np.abs(host(dl).sum(1)) < 1e-5)


def test_softmax_ce_rejects_bad_label_on_device(P):
    L = torch.zeros((2, 4225), dtype=torch.float32, device="cuda")
    loss = torch.empty(2, dtype=torch.float32, device="cuda")
    dl = torch.empty_like(L)
    P.lp_softmax_ce(L, torch.tensor([4225, 3], dtype=torch.int32, device="cuda"), loss, dl)
    torch.cuda.synchronize()
    lo = loss.cpu().numpy()
    assert np.isnan(lo[0]) and np.isclose(lo[1], np.log(4225.0), rtol=1e-6)


def test_head_backward(P):
    rng = np.random.default_rng(9)
    B = 2
    a3 = rand_act(rng, (B, 32, 64, 64))
    wh = cnn.to_f32(rng.standard_normal(32) * 0.2).astype(np.float64)
    dl = cnn.to_f32(rng.standard_normal((B, 65, 65)) * 1e-4).astype(np.float64)
    ds_ref = cnn.sample_transpose(dl)
    ds_mag = cnn.sample_transpose(np.abs(dl))
    dz_exact = np.einsum("byx,c->bcyx", ds_ref, wh) * (a3 > 0)
    dwh_ref = np.einsum("byx,bcyx->c", ds_ref, a3)
    dbh_ref = ds_ref.sum()
    ds = torch.empty((B, 64, 64), dtype=torch.float32, device="cuda")
    dz3 = torch.empty(a3.shape, dtype=torch.bfloat16, device="cuda")
    dwh = torch.empty(32, dtype=torch.float32, device="cuda")
    dbh = torch.empty(1, dtype=torch.float32, device="cuda")
    P.lp_head_bwd(torch.tensor(dl, dtype=torch.float32, device="cuda"), bf(a3),
                  torch.tensor(wh, dtype=torch.float32, device="cuda"), ds, dz3, dwh, dbh)
    torch.cuda.synchronize()
    g_ds = host(ds)
    assert np.all(np.abs(g_ds - ds_ref) <= 10 * U * ds_mag)
    # dz3 = bf16(ds_gpu * wh): bracket the product of the exact ds and wh
    bound = (10 * U * ds_mag + U * np.abs(ds_ref)) [:, None] * np.abs(wh)[None, :, None, None] + 0.0
    bound = np.broadcast_to(bound, dz_exact.shape) * (a3 > 0)
    bracket(host(dz3), dz_exact, bound + 1e-30)
    n = B * 64 * 64
    mag = np.einsum("byx,bcyx->c", np.abs(g_ds), a3)
    assert np.all(np.abs(host(dwh) - np.einsum("byx,bcyx->c", g_ds, a3)) <= n * U * mag + 1e-30)
    assert np.linalg.norm(host(dwh) - dwh_ref) <= 1e-3 * np.linalg.norm(dwh_ref)
    assert abs(host(dbh)[0] - dbh_ref) <= n * U * np.abs(g_ds).sum() + 1e-6 * abs(dbh_ref)


def test_crop(P):
    rng = np.random.default_rng(10)
    feat = rng.integers(0, 256, (7, 150, 211), dtype=np.uint8)
    centers = np.array([[75, 105], [0, 0], [149, 210], [64, 64], [-100, 400]], np.int32)
    x = torch.empty((5, 7, 128, 128), dtype=torch.bfloat16, device="cuda")
    P.lp_crop(torch.from_numpy(feat).cuda(), torch.from_numpy(centers).cuda(), x)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(x), cnn.crop(feat, centers))


def test_crop_from_frame_stack(P):
    rng = np.random.default_rng(11)
    stack = rng.integers(0, 256, (3, 7, 90, 120), dtype=np.uint8)
    frames = np.array([2, 0, 1, 3, -1], np.int32)          # the last two are outside the stack: zeros
    centers = np.array([[45, 60], [10, 100], [80, 5], [45, 60], [45, 60]], np.int32)
    x = torch.empty((5, 7, 64, 64), dtype=torch.bfloat16, device="cuda")
    P.lp_crop(torch.from_numpy(stack).cuda(), torch.from_numpy(centers).cuda(), x, side=64,
              frames=torch.from_numpy(frames).cuda())
    torch.cuda.synchronize()
    g = host(x)
    for b in range(3):
        np.testing.assert_array_equal(g[b], cnn.crop(stack[frames[b]], centers[b:b + 1], side=64)[0])
    assert np.all(g[3:] == 0)


def test_origins(P):
    base = torch.tensor([[100, 200], [5, 7]], dtype=torch.int32, device="cuda")
    allo = P.lp_origins(base).cpu().numpy().reshape(2, 65, 65, 2)
    dy, dx = np.meshgrid(np.arange(-32, 33), np.arange(-32, 33), indexing="ij")
    np.testing.assert_array_equal(allo[0, ..., 0], 100 + dy)
    np.testing.assert_array_equal(allo[1, ..., 1], 7 + dx)
    idx = torch.tensor([[0, 4224, 2112], [65, -1, 4225]], dtype=torch.int32, device="cuda")
    o = P.lp_origins(base, idx=idx).cpu().numpy().reshape(2, 3, 2)
    assert o[0].tolist() == [[68, 168], [132, 232], [100, 200]]
    assert o[1, 0].tolist() == [5 - 31, 7 - 32]
    assert np.all(o[1, 1:] < -(1 << 29))


def test_pack_layout(P):
    p = cnn.init_params(3)
    net = P.ProposalNet(p, max_batch=1)
    net.pack()
    torch.cuda.synchronize()
    W1, W2, W3 = (cnn.bf16(p[k]) for k in ("W1", "W2", "W3"))
    np.testing.assert_array_equal(host(net.w1).reshape(32, 72), pack_w(W1))
    np.testing.assert_array_equal(host(net.w2).reshape(32, 288), pack_w(W2))
    np.testing.assert_array_equal(host(net.w3).reshape(32, 288), pack_w(W3))
    np.testing.assert_array_equal(host(net.w2t).reshape(32, 288), pack_w(flip_t(W2)))
    np.testing.assert_array_equal(host(net.w3t).reshape(32, 288), pack_w(flip_t(W3)))
    got = net.get_params()
    for k in p:
        np.testing.assert_array_equal(got[k], p[k])


@pytest.mark.parametrize("n,k", [(4225, 64), (4225, 1), (8192, 1024), (37, 37), (1000, 200)])
def test_topk(P, n, k):
    rng = np.random.default_rng(12 + n + k)
    L = cnn.to_f32(rng.standard_normal((5, n))).astype(np.float64)
    L[1, n // 10: n // 10 + n // 5] = 5.0      # a wide tie at the top: lower indices first
    L[2, :] = 0.0                              # everything tied
    L[2, ::3] = -0.0                           # -0 ranks with +0
    L[3] = np.round(L[3], 1)                   # many small ties across the threshold
    L[4, :] = 1e-30 * np.arange(n)[::-1]       # tiny distinct values
    idx = P.lp_topk(torch.tensor(L, dtype=torch.float32, device="cuda"), k)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(idx.cpu().numpy(), cnn.topk(L, k))


def test_topk_nan_last(P):
    L = np.array([[1.0, np.nan, 3.0, np.nan, 2.0]])
    idx = P.lp_topk(torch.tensor(L, dtype=torch.float32, device="cuda"), 5)
    assert idx.cpu().numpy().tolist() == [[2, 4, 0, 1, 3]]


def test_sgd(P):
    rng = np.random.default_rng(13)
    n = 20577
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    v = rng.standard_normal(n).astype(np.float32)
    pt, gt, vt = (torch.from_numpy(a.copy()).cuda() for a in (p, g, v))
    P.lp_sgd(pt, gt, vt, 0.05, 0.9, 1e-4)
    torch.cuda.synchronize()
    p2, v2 = cnn.sgd_step({"a": p}, {"a": g}, {"a": v}, 0.05, 0.9, 1e-4)
    # FP32 evaluation of three operations: a few ulps of the operands' magnitude
    assert np.all(np.abs(vt.cpu().numpy() - v2["a"]) <= 4 * 2.0 ** -23 * (np.abs(v) + np.abs(g) + 1))
    assert np.all(np.abs(pt.cpu().numpy() - p2["a"]) <= 4 * 2.0 ** -23 * (np.abs(p) + 1))


def test_network_end_to_end(P):
    """Whole forward and backward pass against the oracle with BF16 rounding at
    the same points; inputs are a smooth feature-like crop."""
    rng = np.random.default_rng(14)
    params = cnn.init_params(21)
    params = {k: (v + (0.02 * rng.standard_normal(v.shape) if k.startswith("b") else 0)).astype(np.float32)
              for k, v in params.items()}
    B = 2
    feat = (np.stack([smooth(rng, 180, 200, 9) for _ in range(7)]) * 255).astype(np.uint8)
    centers = np.array([[90, 100], [60, 130]], np.int32)
    labels = np.array([cnn.NOFF * 30 + 40, cnn.NOFF * 50 + 2])
    x_ref = cnn.crop(feat, centers)
    loss_ref, g_ref, logits_ref = cnn.loss_and_grads(params, x_ref, labels)
    net = P.ProposalNet(params, max_batch=4)
    x = net.crop(torch.from_numpy(feat).cuda(), torch.from_numpy(centers).cuda())
    logits = net.forward(x)
    loss = net.backward(x, torch.tensor(labels, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(x), x_ref)
    lg = host(logits)
    assert np.linalg.norm(lg - logits_ref) <= 1e-3 * np.linalg.norm(logits_ref)
    assert abs(host(loss).mean() - loss_ref) <= 1e-3 * abs(loss_ref)
    g = net.get_params(net.grads)
    # the head bias gradient is the sum of (softmax - onehot), zero up to rounding
    assert abs(g["bh"][0]) <= 1e-6 and abs(g_ref["bh"][0]) <= 1e-12
    errs = {k: np.linalg.norm(g[k] - g_ref[k]) / np.linalg.norm(g_ref[k]) for k in g_ref if k != "bh"}
    print(" ".join("%s %.2e" % kv for kv in errs.items()))
    assert max(errs.values()) <= 1e-3, errs


def test_training_is_deterministic_and_resumable(P):
    rng = np.random.default_rng(15)
    feat = (np.stack([smooth(rng, 200, 220, 6) for _ in range(7)]) * 255).astype(np.uint8)
    ft = torch.from_numpy(feat).cuda()
    centers = torch.tensor([[100, 110], [80, 90], [120, 130]], dtype=torch.int32, device="cuda")
    labels = torch.tensor([2112, 100, 4000], dtype=torch.int32, device="cuda")
    p0 = cnn.init_params(4)

    def run(net, steps):
        losses = []
        for _ in range(steps):
            x = net.crop(ft, centers)
            losses.append(net.train_step(x, labels, lr=0.05).mean().item())
        return losses

    a = P.ProposalNet(p0, max_batch=3)
    la = run(a, 4)
    b = P.ProposalNet(p0, max_batch=3)
    run(b, 2)
    st = b.state()
    c = P.ProposalNet(cnn.init_params(99), max_batch=3)
    c.load_state(st)
    lc = run(c, 2)
    assert torch.equal(a.params, c.params) and torch.equal(a.mom, c.mom)
    assert la[2:] == lc
    assert la[-1] < la[0]
