"""Model of the column-stream write-out's row prefix (planes-innermost frames
of at most 32 planes): the 64 lanes of a wavefront are S = 64 / P2 streams of
P2 planes (lane = stream * P2 + plane), each owning TW / S consecutive columns
of the tile; every stream counts its run's hits, an inclusive scan across the
streams reads the value d * P2 lanes below for d = 1, 2, 4, ... (taken only
when the stream index is at least d), and the run's prefix starts from the
exclusive part.  Checked against the plain running sum of each plane's row."""
import numpy as np
import pytest


def stream_prefix(hits, S):
    """hits: P2 x TW 0/1 (or weights) per plane and column; returns the per-column
    row prefix of every plane as the lanes compute it."""
    P2, TW = hits.shape
    L = TW // S
    lanes = 64
    seg = np.zeros(lanes, np.int64)
    for lane in range(lanes):
        q, p = divmod(lane, P2)
        seg[lane] = hits[p, q * L:(q + 1) * L].sum()
    incl = seg.copy()
    d = 1
    while d < S:
        src = incl[[(lane - d * P2) & 63 for lane in range(lanes)]]
        q = np.arange(lanes) // P2
        incl = incl + np.where(q >= d, src, 0)
        d <<= 1
    out = np.zeros((P2, TW), np.int64)
    for lane in range(lanes):
        q, p = divmod(lane, P2)
        run = incl[lane] - seg[lane]
        for i in range(L):
            run += hits[p, q * L + i]
            out[p, q * L + i] = run
    return out


@pytest.mark.parametrize("S", [2, 4, 8])
@pytest.mark.parametrize("TW", [16, 32])
def test_stream_prefix_equals_running_sum(S, TW):
    rng = np.random.default_rng(S * 100 + TW)
    P2 = 64 // S
    for _ in range(20):
        hits = rng.integers(0, 3, size=(P2, TW))
        assert np.array_equal(stream_prefix(hits, S), np.cumsum(hits, axis=1))
