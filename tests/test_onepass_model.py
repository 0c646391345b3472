"""CPU model of the single-pass build's band algorithm and look-back protocol
(row bands walked tile by tile; per tile a local aggregate in integral form,
a look-back over the bands above through published aggregates and inclusive
bottom rows; row carries kept per band).  Workers are coroutines run in random
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


def model_build(img, bins, bits, R, TW, PG, patience, resident, seed, moments=True):
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
        lc = np.zeros((rows, PG), np.int64)     # row carries (count) left of the tile
        lcy = np.zeros((rows, PG), np.int64)    # row carries (column moment)
        lcs = np.zeros(PG, np.int64)            # sum_r lc
        lcxs = np.zeros(PG, np.int64)           # sum_r r * lc
        lcys = np.zeros(PG, np.int64)           # sum_r lcy
        for j in range(nT):
            C0, C1 = j * TW, min(W, (j + 1) * TW)
            cb = binned[ch, R0:R0 + rows, C0:C1] - kb          # rows x tile cols
            rr = np.arange(R0, R0 + rows, dtype=np.int64)[:, None]
            hit = np.stack([(cb == k) for k in range(PG)]).astype(np.int64)  # PG x rows x cols
            cnt = hit.sum(1)
            cntx = (hit * rr).sum(1)
            A = lcs[:, None] + np.cumsum(cnt, 1)
            AX = lcxs[:, None] + np.cumsum(cntx, 1)
            AY = lcys[:, None] + np.cumsum(cnt * cols[C0:C1], 1)
            top = np.zeros((3, PG, C1 - C0), np.int64)
            if b > 0:
                polls = 0
                while flags.get((b - 1, gi, j), 0) == 0 and (patience < 0 or polls < patience):
                    polls += 1
                    yield
                if flags.get((b - 1, gi, j), 0) != 2:
                    if b != nB - 1:
                        agg[(b, gi, j)] = np.stack([A, AX, AY])
                        flags[(b, gi, j)] = 1
                    bb = b - 1
                    while True:
                        while flags.get((bb, gi, j), 0) == 0:
                            yield
                        if flags[(bb, gi, j)] == 2:
                            top += inc[(bb, gi, j)]
                            break
                        top += agg[(bb, gi, j)]
                        bb -= 1
                        assert bb >= 0
                else:
                    top += inc[(b - 1, gi, j)]
            if b != nB - 1:
                inc[(b, gi, j)] = top + np.stack([A, AX, AY])
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
            lcs = lc.sum(0)
            lcxs = (np.arange(R0, R0 + rows)[:, None] * lc).sum(0)
            lcys = lcy.sum(0)
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
    # C, H, W, bins, bits, R, TW, PG, patience, resident
    (1, 37, 50, 5, 8, 4, 8, 2, -1, 3),
    (2, 23, 41, 3, 8, 1, 8, 1, 0, 50),
    (1, 40, 29, 8, 16, 7, 16, 4, 2, 5),
    (3, 16, 16, 4, 8, 16, 8, 2, 0, 1),
    (1, 64, 33, 6, 8, 3, 8, 4, 1, 200),
]


@pytest.mark.parametrize("case", CASES)
def test_band_lookback_model_matches_oracle(case):
    C, H, W, bins, bits, R, TW, PG, patience, resident = case
    rng = np.random.default_rng(sum(case))
    img = rng.integers(0, 1 << bits, size=(C, H, W)).astype(np.uint8 if bits <= 8 else np.uint16)
    ref = oracle.ih(img, bins, bits)
    omx, omy = oracle.moments(img, bins, bits)
    for seed in range(3):
        out, mx, my = model_build(img, bins, bits, R, TW, PG, patience, resident, seed)
        assert np.array_equal(out, ref)
        assert np.array_equal(mx & M32, np.asarray(omx).astype(np.int64) & M32)
        assert np.array_equal(my & M32, np.asarray(omy).astype(np.int64) & M32)
