"""CPU model of the single-pass build's band algorithm and look-back protocol
(row bands swept twice: first every tile's band aggregate in integral form,
published without waiting; then per tile a look-back over the bands above to
the nearest published inclusive bottom row through the aggregates in between,
inspected a chunk of bands at a time, and the write-out with row carries kept
per band).  Workers are coroutines run in random
interleavings with a bounded number resident at once and tickets handed out
in start order; the model's integral histogram and moment tensors must equal
the oracle's, and no interleaving may deadlock.  This pins the arithmetic the
GPU kernel implements (integral-form aggregates, the band sums of the row
carries and the moment terms), independently of the GPU."""
import random

import numpy as np
import pytest

import oracle

M32 = 0xFFFFFFFF


def model_build(img, bins, bits, R, TW, PG, patience, resident, seed, lanes=64, moments=True):
    C, H, W = img.shape
    P = C * bins
    nB, nT = -(-H // R), -(-W // TW)
    gpc = -(-bins // PG)
    nG = C * gpc
    binned = ((img.astype(np.uint64) * bins) >> bits).astype(np.int64)
    out = np.zeros((P, H, W), np.int64)
    mx = np.zeros((P, H, W), np.int64)
    my = np.zeros((P, H, W), np.int64)
    flags = {}            # (band, group, tile) -> 1 (aggregate) / 2 (inclusive)
    agg, inc = {}, {}     # payloads: arrays of (k, column) for counts, row moments, column moments
    cols = np.arange(W, dtype=np.int64)

    def worker(t):
        b, gi = divmod(t, nG)
        ch, kb = gi // gpc, (gi % gpc) * PG
        nk = min(PG, bins - kb)
        R0 = b * R
        rows = min(R, H - R0)
        rr = np.arange(R0, R0 + rows, dtype=np.int64)[:, None]
        last = b == nB - 1
        # sweep A: every tile's band aggregate, published without waiting
        lcs = np.zeros(PG, np.int64)            # band counts left of the tile
        lcxs = np.zeros(PG, np.int64)           # their row moments
        lcys = np.zeros(PG, np.int64)           # their column moments
        for j in range(nT):
            C0, C1 = j * TW, min(W, (j + 1) * TW)
            cb = binned[ch, R0:R0 + rows, C0:C1] - kb
            hit = np.stack([(cb == k) for k in range(PG)]).astype(np.int64)  # PG x rows x cols
            cnt = hit.sum(1)
            cntx = (hit * rr).sum(1)
            A = np.stack([lcs[:, None] + np.cumsum(cnt, 1), lcxs[:, None] + np.cumsum(cntx, 1),
                          lcys[:, None] + np.cumsum(cnt * cols[C0:C1], 1)])
            if not last:
                if b == 0:
                    inc[(b, gi, j)] = A
                    flags[(b, gi, j)] = 2
                else:
                    agg[(b, gi, j)] = A
                    flags[(b, gi, j)] = 1
            lcs = lcs + cnt.sum(1)
            lcxs = lcxs + cntx.sum(1)
            lcys = lcys + (cnt * cols[C0:C1]).sum(1)
            yield
        # sweep B: top boundary from the nearest inclusive row above plus the
        # aggregates in between (flags inspected `lanes` bands at a time), then
        # the write-out with row carries
        lc = np.zeros((rows, PG), np.int64)
        lcy = np.zeros((rows, PG), np.int64)
        for j in range(nT):
            C0, C1 = j * TW, min(W, (j + 1) * TW)
            cb = binned[ch, R0:R0 + rows, C0:C1] - kb
            hit = np.stack([(cb == k) for k in range(PG)]).astype(np.int64)
            top = np.zeros((3, PG, C1 - C0), np.int64)
            if b > 0:
                for _ in range(max(patience, 0)):
                    if flags.get((b - 1, gi, j), 0) == 2:
                        break
                    yield
                hi = b - 1
                while True:
                    assert hi >= 0                  # band 0 always ends the walk
                    chunk = list(range(hi, max(hi - lanes, -1), -1))
                    while True:
                        f = [flags.get((x, gi, j), 0) for x in chunk]
                        near = f.index(2) if 2 in f else None
                        cover = f[:near + 1] if near is not None else f
                        if 0 not in cover:
                            break
                        yield
                    n_agg = near if near is not None else len(chunk)
                    for x in chunk[:n_agg]:
                        top += agg[(x, gi, j)]
                    if near is not None:
                        top += inc[(chunk[near], gi, j)]
                        break
                    hi -= lanes
                if not last:
                    inc[(b, gi, j)] = top + agg[(b, gi, j)]
                    flags[(b, gi, j)] = 2
            col, colx, coly = top[0].copy(), top[1].copy(), top[2].copy()
            for r in range(rows):
                pre = lc[r][:, None] + np.cumsum(hit[:, r, :], 1)
                ypre = lcy[r][:, None] + np.cumsum(hit[:, r, :] * cols[C0:C1], 1)
                col += pre
                colx += (R0 + r) * pre
                coly += ypre
                for k in range(nk):
                    p = ch * bins + kb + k
                    out[p, R0 + r, C0:C1] = col[k]
                    mx[p, R0 + r, C0:C1] = colx[k]
                    my[p, R0 + r, C0:C1] = coly[k]
                lc[r] = pre[:, -1]
                lcy[r] = ypre[:, -1]
            yield

    rng = random.Random(seed)
    n = nB * nG
    ticket, running, active = 0, [], {}
    while ticket < n or running:
        while len(running) < resident and ticket < n:
            active[ticket] = worker(ticket)
            running.append(ticket)
            ticket += 1
        t = rng.choice(running)
        try:
            next(active[t])
        except StopIteration:
            running.remove(t)
    return out, mx, my


CASES = [
    # C, H, W, bins, bits, R, TW, PG, patience, resident, lanes (bands per flag read)
    (1, 37, 50, 5, 8, 4, 8, 2, -1, 3, 64),
    (2, 23, 41, 3, 8, 1, 8, 1, 0, 50, 4),
    (1, 40, 29, 8, 16, 7, 16, 4, 2, 5, 2),
    (3, 16, 16, 4, 8, 16, 8, 2, 0, 1, 64),
    (1, 64, 33, 6, 8, 3, 8, 4, 1, 200, 3),
    (1, 70, 20, 2, 8, 1, 8, 1, 0, 400, 1),
]


@pytest.mark.parametrize("case", CASES)
def test_band_lookback_model_matches_oracle(case):
    C, H, W, bins, bits, R, TW, PG, patience, resident, lanes = case
    rng = np.random.default_rng(sum(case))
    img = rng.integers(0, 1 << bits, size=(C, H, W)).astype(np.uint8 if bits <= 8 else np.uint16)
    ref = oracle.ih(img, bins, bits)
    omx, omy = oracle.moments(img, bins, bits)
    for seed in range(3):
        out, mx, my = model_build(img, bins, bits, R, TW, PG, patience, resident, seed, lanes)
        assert np.array_equal(out, ref)
        assert np.array_equal(mx & M32, np.asarray(omx).astype(np.int64) & M32)
        assert np.array_equal(my & M32, np.asarray(omy).astype(np.int64) & M32)
