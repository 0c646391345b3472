"""ih_build_noalloc (the build on the library's per-GPU scratch array, for
callers that cannot allocate) against ih_build with a caller workspace, both
called through the C ABI: bit-identical integral histograms and moment
tensors in both layouts and both pass counts, on consecutive calls whose
second input is smaller, the status word, and the refusal of shapes whose
workspace exceeds the scratch array."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
P_ = ctypes.c_void_p


def ihlib():
    import paper_1711_01656_amd as ih
    return ih


def say(*a):
    print(*a, flush=True)


def ptr(t):
    return P_(t.data_ptr()) if t is not None else P_(0)


def rand_img(seed, C, H, W, bits):
    rng = np.random.default_rng(seed)
    dt = np.uint8 if bits <= 8 else np.uint16
    return torch.from_numpy(rng.integers(0, 1 << bits, size=(C, H, W)).astype(dt)).to(DEV)


def shape(P, H, W, layout):
    return (P, H, W) if layout == 0 else (H, W, P)


def both(img, bins, bits, layout, moments, cfg):
    """(with-workspace result, allocation-free result, status word) of one shape."""
    ih = ihlib()
    L = ih.lib()
    C, H, W = img.shape
    dt = 0 if img.dtype == torch.uint8 else 1
    P = C * bins
    shp = shape(P, H, W, layout)
    cfgp = ctypes.byref(cfg) if cfg is not None else None
    ref = [torch.full(shp, -3, dtype=torch.int32, device=DEV) for _ in range(3 if moments else 1)]
    got = [torch.full(shp, -5, dtype=torch.int32, device=DEV) for _ in range(3 if moments else 1)]
    wsb = L.ih_build_workspace_size(H, W, C, bins, int(moments), layout, cfgp)
    assert wsb > 0, L.ih_last_error()
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    mx = ref[1] if moments else None
    my = ref[2] if moments else None
    rc = L.ih_build(ptr(img), dt, H, W, C, bins, bits, layout, ptr(ref[0]), ptr(mx), ptr(my), cfgp, ptr(ws),
                    wsb, None)
    assert rc == 0, L.ih_last_error()
    status = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    mx = got[1] if moments else None
    my = got[2] if moments else None
    rc = L.ih_build_noalloc(ptr(img), dt, H, W, C, bins, bits, layout, ptr(got[0]), ptr(mx), ptr(my), cfgp,
                            ptr(status), None)
    assert rc == 0, L.ih_last_error()
    torch.cuda.synchronize()
    return ref, got, int(status.item())


CASES = [
    # (C, H, W, bins, bits, layout, moments, cfg) pairs: a call, then a smaller one
    ("bhw three-pass u8 + moments", (1, 300, 517, 16, 8, 0, True, None), (1, 97, 203, 8, 8, 0, True, None)),
    ("hwb three-pass u16", (2, 211, 333, 32, 16, 1, False, None), (1, 64, 77, 8, 16, 1, False, None)),
    ("hwb three-pass u8 + moments", (7, 120, 260, 16, 8, 1, True, None), (3, 50, 64, 16, 8, 1, True, None)),
    ("bhw single-pass u16 + moments", (1, 400, 700, 64, 16, 0, True, (64, 256, 1)),
     (1, 130, 301, 5, 16, 0, True, (32, 128, 2))),
    ("bhw single-pass u8", (3, 257, 513, 32, 8, 0, False, (16, 128, 4)), (1, 33, 65, 4, 8, 0, False, (7, 64, 1))),
]


@pytest.mark.parametrize("name,first,second", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_ih_build_twice(name, first, second):
    ih = ihlib()
    for k, (C, H, W, bins, bits, layout, moments, c) in enumerate((first, second)):
        say(name, "call", k, (C, H, W, bins, bits, layout, moments, c))
        cfg = ih.TileCfg(c[0], c[1], c[2], 1) if c is not None else None
        img = rand_img(1000 * k + H + W, C, H, W, bits)
        ref, got, st = both(img, bins, bits, layout, moments, cfg)
        assert st == 0
        for r, g in zip(ref, got):
            assert torch.equal(r, g), name


def test_noalloc_status_and_stale_scratch():
    """A value beyond value_bits sets the status bit; the next clean call on
    the same scratch array reports 0 again (the build clears it)."""
    ih = ihlib()
    img = rand_img(5, 1, 50, 70, 6)
    bad = img.clone()
    bad[0, 17, 33] = 200
    for cfg in (None, ih.TileCfg(16, 64, 2, 1)):
        say("status", cfg)
        _, _, st = both(img, 8, 6, 0, False, cfg)
        assert st == 0
        _, _, st = both(bad, 8, 6, 0, False, cfg)
        assert st & ih.STATUS_VALUE_RANGE
        ref, got, st = both(img, 8, 6, 0, False, cfg)
        assert st == 0 and torch.equal(ref[0], got[0])


def test_noalloc_refuses_shapes_beyond_the_scratch():
    ih = ihlib()
    L = ih.lib()
    H, W, bins = 6144, 4096, 64
    need = L.ih_build_workspace_size(H, W, 1, bins, 0, 0, None)
    assert need > ih.NOALLOC_SCRATCH_BYTES
    img = torch.zeros((1, H, W), dtype=torch.uint8, device=DEV)
    out = torch.full((bins, H, W), 7, dtype=torch.int32, device=DEV)   # full size, so nothing can go out of bounds
    rc = L.ih_build_noalloc(ptr(img), 0, H, W, 1, bins, 8, 0, ptr(out), None, None, None, None, None)
    assert rc == -6 and b"scratch" in L.ih_last_error()
    torch.cuda.synchronize()
    assert bool((out[:, ::97, ::89] == 7).all())       # the refused call enqueued nothing
    del out
    torch.cuda.empty_cache()
