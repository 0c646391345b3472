"""Model of the strip write-out's row windows (bin-major rows that do not
start on 64-byte boundaries): a wave walks a strip of tiles of width TW = 64
CPL; tile t's row goes out as the window [C0 - d, C0 + TW - d) (the strip's
first tile from C0, its last tile up to min(C0 + TW, W)), d being the row's
misalignment in ints, through a ring of 2 TW slots holding column c at
(c + d) mod 2 TW.  Checked for random shapes and row offsets: every column of the row is
written exactly once, whole 4-int groups start on 16-byte boundaries, every
slot a window reads holds the column it stands for, and the slots a tile
writes are never ones a later window of the same row still needs."""
import numpy as np
import pytest


def row_windows(W, CPL, G, base):
    """base: the row's column 0 in ints past a 64-byte boundary."""
    TW = 64 * CPL
    RING = 2 * TW
    nTC = -(-W // TW)
    writes = np.zeros(W, np.int64)
    ring = {}
    for j0 in range(0, nTC, G):
        nt = min(G, nTC - j0)
        for t in range(nt):
            C0 = (j0 + t) * TW
            d = (base + C0) % 16                      # the kernel's misalignment of column C0
            for x in range(TW):                       # the tile's row into the ring
                ring[(C0 + x + d) % RING] = C0 + x
            wlo = C0 if t == 0 else C0 - d
            whi = min(C0 + TW, W) if t == nt - 1 else C0 + TW - d
            for q in range((TW + 16) // 4):
                c = C0 - d + 4 * q
                if not (c < whi and c + 4 > wlo):
                    continue
                slot = (C0 + 4 * q) % RING
                assert slot % 4 == 0
                full = c >= wlo and c + 4 <= whi
                if full:
                    assert (base + c) % 4 == 0         # a 16-byte store on a 16-byte boundary
                    if q == 0:
                        assert (base + c) % 16 == 0    # the window's first group on a 64-byte boundary
                for i in range(4):
                    if wlo <= c + i < whi:
                        assert ring[slot + i] == c + i, (c + i, ring[slot + i])
                        writes[c + i] += 1
    return writes


@pytest.mark.parametrize("seed", range(40))
def test_every_column_once_and_ring_consistent(seed):
    rng = np.random.default_rng(seed)
    CPL = int(rng.choice([1, 2, 4]))
    PG = int(rng.choice([1, 2, 4, 8, 16]))
    G = max(1, 16 // (CPL * PG))
    W = int(rng.integers(1, 5 * 64 * CPL * G))
    base = int(rng.integers(0, 1 << 20))
    writes = row_windows(W, CPL, G, base)
    assert np.all(writes == 1), np.nonzero(writes != 1)[0][:10]


def test_aligned_row_and_single_tile_strips():
    for CPL in (1, 2, 4):
        for W in (64 * CPL, 64 * CPL * 3 + 7, 1):
            assert np.all(row_windows(W, CPL, 1, 5) == 1)
            assert np.all(row_windows(W, CPL, 4, 0) == 1)
            assert np.all(row_windows(W, CPL, 4, 1023) == 1)
