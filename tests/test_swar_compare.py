"""The byte-parallel equality test the register tile pass uses to compare
four staged bins (the bytes of a word) with one bin k: with lo = the word's
low seven bits per byte, hi = its top bits flipped to mean "equal to k's top
bit", hi & ~((lo ^ key) + 0x7f7f7f7f) holds 0x80 exactly in the bytes equal
to k.  Checked here for every byte value against every bin, with random
neighbouring bytes (no carry may cross a byte)."""
import numpy as np

M = 0xFFFFFFFF


def swar_match(words, k):
    key = (k & 0x7F) * 0x01010101
    flip = 0 if (k & 0x80) else 0x80808080
    lo = words & 0x7F7F7F7F
    hi = (words & 0x80808080) ^ flip
    return hi & (~((lo ^ key) + 0x7F7F7F7F) & M)


def test_every_byte_against_every_bin():
    rng = np.random.default_rng(0)
    for k in range(256):
        b = rng.integers(0, 256, size=(2048, 4), dtype=np.uint64)
        for e in range(4):
            b[256 * e:256 * (e + 1), e] = np.arange(256)
        w = b[:, 0] | (b[:, 1] << 8) | (b[:, 2] << 16) | (b[:, 3] << 24)
        m = swar_match(w, k)
        for e in range(4):
            assert np.array_equal((m >> (8 * e + 7)) & 1, (b[:, e] == k).astype(np.uint64))
            assert not np.any((m >> (8 * e)) & 0x7F)


def test_byte_counters_and_bit_counts():
    """Column counts as byte lanes (flags >> 7 summed over up to 128 rows)
    and row counts as bit counts equal direct counting."""
    rng = np.random.default_rng(1)
    for k in (0, 5, 127, 128, 200, 255):
        b = rng.choice([k, (k + 1) % 256, 0, 255], size=(128, 4)).astype(np.uint64)
        w = b[:, 0] | (b[:, 1] << 8) | (b[:, 2] << 16) | (b[:, 3] << 24)
        m = swar_match(w, k)
        acc = int(np.sum(m >> 7))
        for e in range(4):
            assert (acc >> (8 * e)) & 0xFF == int(np.sum(b[:, e] == k)) % 256
        rows = [bin(int(x)).count("1") for x in m]
        assert rows == [int(np.sum(r == k)) for r in b]


def test_moment_sums_from_match_flags():
    """Coordinate moments from the same flags: per column, the tile-local row
    index summed in two 16-bit halves (columns 0 and 2, columns 1 and 3) of
    the flags times the row, over up to 256 rows; per word of a row, the
    matching bytes' offsets e from byte 2 of the 24-bit product of the flags
    of bytes 1-3 with 0x010203.  Both equal direct sums, with every step in
    32-bit arithmetic as on the device."""
    rng = np.random.default_rng(2)
    for k in (0, 3, 127, 128, 255):
        for th in (1, 7, 128, 129, 256):
            b = rng.choice([k, k ^ 1, k ^ 0x80, 0], size=(th, 4), p=[0.7, 0.1, 0.1, 0.1]).astype(np.uint64)
            if k == 0:
                b[:] = k  # every byte matches: the halves' largest sums
            w = b[:, 0] | (b[:, 1] << 8) | (b[:, 2] << 16) | (b[:, 3] << 24)
            ax02 = ax13 = 0
            for r in range(th):
                m = int(swar_match(w[r], k)) >> 7
                ax02 = (ax02 + (m & 0x00010001) * r) & M
                ax13 = (ax13 + (((m >> 8) & 0x00010001) * r)) & M
            direct = [int(np.sum(np.arange(th)[b[:, e] == k])) for e in range(4)]
            assert [ax02 & 0xFFFF, ax13 & 0xFFFF, ax02 >> 16, ax13 >> 16] == direct
            for r in range(th):
                m = int(swar_match(w[r], k))
                u = m >> 15
                assert u < (1 << 24)
                prod = (u * 0x010203) & M  # low 32 bits, as the 24-bit multiply returns
                offs = (prod >> 16) & 0xFF
                assert offs == sum(e for e in range(4) if b[r, e] == k)
