"""The C-ABI library loads and exports every symbol include/*.h declares;
host-side argument checks return error codes without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ih_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_1711_01656_amd as pkg
    from paper_1711_01656_amd import build as hipbuild
    if not os.path.exists(pkg.lib_path()):
        hipbuild.build()
    return pkg.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("ih_build", "ih_query_rect", "ih_query_weighted", "ih_match_candidates",
              "ih_pyramid_desc", "ih_build_workspace_size", "ih_last_error", "ih_version"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_symbol():
    from paper_1711_01656_amd import ih
    assert set(declared_functions()) == set(ih.SIGNATURES)


def test_version_and_error(lib):
    assert lib.ih_version() >= 100
    assert isinstance(lib.ih_last_error(), bytes)


def test_workspace_size_host_only(lib):
    from paper_1711_01656_amd import ih
    n = ih.workspace_size(480, 640, 1, 32)
    assert n > 0
    m = ih.workspace_size(480, 640, 1, 32, moments=True)
    assert m > n
    # carries are a small fraction of the 39 MB integral histogram
    assert n < 0.2 * 480 * 640 * 32 * 4
    assert ih.workspace_size(480, 640, 1, 32, layout="hwb") > 0
    assert lib.ih_build_workspace_size(0, 640, 1, 32, 0, 0, None) == 0
    assert lib.ih_build_workspace_size(480, 640, 1, 300, 0, 0, None) == 0
    assert b"bins" in lib.ih_last_error()
    assert lib.ih_build_workspace_size(480, 640, 1, 32, 0, 5, None) == 0
    assert b"layout" in lib.ih_last_error()


def test_host_argument_errors(lib):
    from paper_1711_01656_amd import ih
    P = ctypes.c_void_p
    fake = P(0x1000)
    big = 1 << 30

    def build(img=fake, dt=0, H=64, W=64, C=1, bins=8, bits=8, layout=0, out=fake, mx=None, my=None,
              cfg=None, ws=fake, wsb=big):
        return lib.ih_build(img, dt, H, W, C, bins, bits, layout, out, mx, my, cfg, ws, wsb, None)

    assert build(img=None) == -1                      # NULL image
    assert build(mx=fake) == -1                       # only one moment pointer
    assert build(dt=7) == -1                          # unknown dtype
    assert build(bits=9) == -1                        # more bits than uint8 holds
    assert build(bins=8, bits=2) == -1                # bins beyond 2^bits
    assert build(layout=3) == -1                      # unknown layout
    assert build(wsb=16) == -6                        # workspace too small
    assert build(ws=None) == -6                       # no workspace
    assert build(H=65536, W=65536) == -3              # H*W beyond int32 counts
    for layout, cfg in ((0, ih.TileCfg(0, 64, 1)), (0, ih.TileCfg(32, 3, 1)), (0, ih.TileCfg(32, 64, 3)),
                        (0, ih.TileCfg(256, 256, 1)), (1, ih.TileCfg(32, 128, 64)), (1, ih.TileCfg(32, 32, 8)),
                        (0, ih.TileCfg(32, 256, 16))):
        mom = fake if cfg.key() == (32, 256, 16) else None
        assert build(layout=layout, cfg=ctypes.byref(cfg), mx=mom, my=mom) < 0, cfg
    # queries
    assert lib.ih_query_rect(fake, 0, 4, 4, 0, fake, 1, fake, None) == -1
    assert lib.ih_query_rect(fake, 2, 4, 4, 0, fake, -1, fake, None) == -1
    assert lib.ih_query_rect(fake, 2, 4, 4, 9, fake, 1, fake, None) == -1
    assert lib.ih_query_rect(None, 2, 4, 4, 0, None, 0, None, None) == 0       # nothing to do
    assert lib.ih_query_weighted(fake, fake, fake, 6, 4, 4, 4, 0, fake, 1, 0, 0, fake, None) == -1
    assert lib.ih_query_weighted(fake, fake, fake, 8, 4, 4, 1, 0, fake, 1, 9, 0, fake, None) == -4
    assert lib.ih_pyramid_desc(fake, 8, 4, 4, 0, fake, 1, 5, fake, None) == -1
    assert lib.ih_match_candidates(fake, 8, 4, 4, 0, fake, 2, 2, 3, fake, 1, 7, fake, fake, None) == -1
    assert lib.ih_match_candidates(fake, 8, 4, 4, 0, fake, 0, 2, 3, fake, 1, 0, fake, fake, None) == -1
    assert lib.ih_match_candidates(fake, 8, 4, 4, 2, fake, 2, 2, 3, fake, 1, 0, fake, fake, None) == -1
    # planes innermost, a pixel row of W*P >= 2^32 entries: refused before any launch
    assert lib.ih_match_candidates(fake, 4096, 1, 1 << 20, 1, fake, 2, 2, 3, fake, 1, 0, fake, fake, None) == -2
    assert b"W*P" in lib.ih_last_error()
    assert lib.ih_profile_events(fake, None) == -1


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1711_01656_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "ih_oracle" not in txt, f


def test_batch_plan_host_only(lib):
    from paper_1711_01656_amd import ih
    n = 3
    arr = (ih.Frame * n)()
    for i, (H, W, bins) in enumerate(((240, 320, 8), (1000, 777, 64), (5, 3, 1))):
        a = arr[i]
        a.img, a.ih = 0x1000, 0x2000
        a.H, a.W, a.C, a.bins, a.value_bits = H, W, 1, bins, 8
    nb = lib.ih_batch_plan_bytes(n)
    assert nb > 0 and lib.ih_batch_plan_bytes(0) == 0
    buf = (ctypes.c_uint8 * nb)()
    ws = ctypes.c_size_t(0)
    assert lib.ih_batch_plan(ctypes.byref(arr), n, 0, 0, buf, nb, ctypes.byref(ws)) == 0
    assert ws.value > 0
    # a search needs its buffers
    arr[0].n_cand = 10
    assert lib.ih_batch_plan(ctypes.byref(arr), n, 0, 0, buf, nb, ctypes.byref(ws)) == -1
    arr[0].origins, arr[0].dist, arr[0].best, arr[0].tmpl_out = 0x3000, 0x4000, 0x5000, 0x6000
    arr[0].win_h = arr[0].win_w = 8
    assert lib.ih_batch_plan(ctypes.byref(arr), n, 0, 0, buf, nb, ctypes.byref(ws)) == 0
    # planes per wave above 8 is refused in a batch; bad dtype, metric, size
    arr[1].tile = ih.TileCfg(32, 64, 16)
    assert lib.ih_batch_plan(ctypes.byref(arr), n, 0, 0, buf, nb, ctypes.byref(ws)) == -4
    arr[1].tile = ih.TileCfg(0, 0, 0)
    assert lib.ih_batch_plan(ctypes.byref(arr), n, 2, 0, buf, nb, ctypes.byref(ws)) == -1
    assert lib.ih_batch_plan(ctypes.byref(arr), n, 0, 5, buf, nb, ctypes.byref(ws)) == -1
    assert lib.ih_batch_plan(ctypes.byref(arr), n, 0, 0, buf, 16, ctypes.byref(ws)) == -1
    # launching an uninitialised plan or with a short workspace is refused
    zero = (ctypes.c_uint8 * nb)()
    assert lib.ih_build_batch(zero, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), 1 << 30, 0, None) == -1
    assert lib.ih_batch_plan(ctypes.byref(arr), n, 0, 0, buf, nb, ctypes.byref(ws)) == 0
    assert lib.ih_build_batch(buf, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), 16, 0, None) == -6
    assert lib.ih_build_batch(buf, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), 1 << 30, 7, None) == -1


def test_onepass_host_checks(lib):
    from paper_1711_01656_amd import ih
    one = ih.onepass(64, 256, 1)
    n = ih.workspace_size(480, 640, 1, 32, cfg=one)
    assert n > 0
    # header + flags + two payload areas of about 1/64 of the output each
    assert n < 0.1 * 480 * 640 * 32 * 4
    assert ih.workspace_size(480, 640, 1, 32, True, cfg=one) > n
    # bad single-pass shapes and layouts are refused on the host
    for bad in (ih.onepass(64, 96, 1), ih.onepass(64, 256, 3), ih.onepass(2000, 256, 1)):
        assert lib.ih_build_workspace_size(480, 640, 1, 32, 0, 0, ctypes.byref(bad)) == 0
    assert lib.ih_build_workspace_size(480, 640, 1, 32, 0, 1, ctypes.byref(one)) == 0
    assert b"bin-major" in lib.ih_last_error()
    big = ih.onepass(1024, 256, 4)   # 64 KB of row carries per block: no room for moments
    assert lib.ih_build_workspace_size(4096, 640, 1, 32, 1, 0, ctypes.byref(big)) == 0
    assert lib.ih_set_lookback_patience(-2) != 0
    assert lib.ih_set_lookback_patience(-1) == 0
    # a three-pass workspace of a shape also fits its single-pass default build
    dflt = ih.workspace_size(1080, 1920, 7, 16, True)
    assert dflt >= lib.ih_build_workspace_size(1080, 1920, 7, 16, 1, 0, ctypes.byref(ih.onepass()))
