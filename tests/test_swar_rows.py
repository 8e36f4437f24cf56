"""Host-only model of the expansion's distance-row test (k_win_expand's
RootRow::direct) in both forms, on random rows: the 8-bit rows (two slots
per 16-bit field, 255 never counting) and the 4-bit copy (byte k of a packed
row holds slot k and slot k + tpad/2, each min(d, 15); a nibble of 15 is
widened to 255).  The 4-bit form must never claim a prune the 8-bit rows do
not (so labels cannot change), and must claim exactly those whose reached
vertex's slot distance is below 15.  Also the prune test's bit-parallel
screen per word (which slots prune by distances alone, which need the sets
for a -1 or -2 correction)."""
import numpy as np
import pytest

M32 = 0xFFFFFFFF


def words(row_bytes):
    """uint8 row -> list of little-endian 32-bit words."""
    b = np.asarray(row_bytes, np.uint8)
    return [int(x) for x in b.view("<u4")]


def sum_hits(aw, bw, D):
    """The SWAR test over one 32-bit word of each row: any byte pair with
    a + b <= D, the sums formed two at a time in 16-bit fields."""
    K = ((D + 1) * 0x00010001) & M32
    hit = 0
    se = (aw & 0x00FF00FF) + (bw & 0x00FF00FF)
    so = ((aw >> 8) & 0x00FF00FF) + ((bw >> 8) & 0x00FF00FF)
    hit |= ~(((se | 0x80008000) - K) & M32) & 0x80008000
    hit |= ~(((so | 0x80008000) - K) & M32) & 0x80008000
    return hit != 0


def pack(row):
    """4-bit copy of an 8-bit row of tpad slots (tpad 32 or 64)."""
    tpad = len(row)
    half = tpad // 2
    lo = np.minimum(np.asarray(row[:half], np.int64), 15)
    hi = np.minimum(np.asarray(row[half:], np.int64), 15)
    return (lo | (hi << 4)).astype(np.uint8)


def unpack_word(w, high):
    c = ((w >> 4) if high else w) & 0x0F0F0F0F
    return c | ((((c + 0x01010101) >> 4) & 0x01010101) * 0xF0)


def direct_full(root, x, D):
    ra, xa = words(root), words(x)
    return any(sum_hits(a, b, D) for a, b in zip(ra, xa))


def direct_packed(root, packed, D):
    half = len(root) // 2
    ra_lo, ra_hi = words(root[:half]), words(root[half:])
    pw = words(packed)
    return any(sum_hits(a, unpack_word(w, False), D) or sum_hits(h, unpack_word(w, True), D)
               for a, h, w in zip(ra_lo, ra_hi, pw))


def exact(root, x, D, cap=255):
    r = np.asarray(root, np.int64)
    v = np.asarray(x, np.int64)
    ok = (r != 255) & (v != 255) & (v < cap)
    return bool(np.any(ok & (r + v <= D)))


@pytest.mark.parametrize("tpad", [32, 64])
def test_four_bit_rows_prune_only_what_the_rows_prune(tpad):
    rng = np.random.default_rng(tpad)
    for it in range(4000):
        # distances mostly small, some saturated, some unreachable (255)
        root = rng.integers(0, 20, tpad)
        x = rng.integers(0, 22, tpad)
        root[rng.random(tpad) < 0.1] = 255
        x[rng.random(tpad) < 0.1] = 255
        D = int(rng.integers(0, 40))
        full = direct_full(root.astype(np.uint8), x.astype(np.uint8), D)
        assert full == exact(root, x, D), (it, D)
        packed = direct_packed(root.astype(np.uint8), pack(x), D)
        assert packed == exact(root, x, D, cap=15), (it, D)
        assert not packed or full  # never a prune the 8-bit rows would not make


def test_saturated_nibble_never_counts():
    root = np.zeros(64, np.uint8)
    x = np.full(64, 15, np.uint8)  # 15 or more
    assert direct_full(root, x, 15)  # the 8-bit rows know 0 + 15 <= 15
    assert not direct_packed(root, pack(x), 254)  # the 4-bit copy claims nothing


def swar_word(aw, bw, D):
    """The prune test's per-word bit-parallel screen (k_win_test): byte
    sums a + c of the root's and the vertex's distances, two at a time in
    16-bit fields; hit when some sum is at most D, and per byte the slots
    whose sum is exactly D + 1 (n2: a -1 or -2 correction would prune) or
    D + 2 (n1: only -2 would), both distances finite."""
    K1 = ((D + 1) * 0x00010001) & M32
    K2 = ((D + 2) * 0x00010001) & M32
    hit = 0
    z1, z2 = [0, 0], [0, 0]
    for h in range(2):
        a = (aw >> (8 * h)) & 0x00FF00FF
        c = (bw >> (8 * h)) & 0x00FF00FF
        s = a + c
        hit |= ~(((s | 0x80008000) - K1) & M32) & 0x80008000
        inf = ((((a + 0x00010001) | (c + 0x00010001)) >> 8) & 0x00010001)
        s |= inf * 0x1FF
        x1, x2 = s ^ K1, s ^ K2
        z1[h] = ~(((x1 | 0x80008000) - 0x00010001) & M32) & 0x80008000
        z2[h] = ~(((x2 | 0x80008000) - 0x00010001) & M32) & 0x80008000
    n2 = ((z1[0] >> 15) & 1) | ((z1[1] >> 14) & 2) | ((z1[0] >> 29) & 4) | ((z1[1] >> 28) & 8)
    n1 = ((z2[0] >> 15) & 1) | ((z2[1] >> 14) & 2) | ((z2[0] >> 29) & 4) | ((z2[1] >> 28) & 8)
    return hit != 0, n1, n2


def test_bit_parallel_screen_words():
    rng = np.random.default_rng(11)
    for it in range(20000):
        a = rng.integers(0, 130, 4)
        c = rng.integers(0, 130, 4)
        a[rng.random(4) < 0.15] = 255
        c[rng.random(4) < 0.15] = 255
        D = int(rng.integers(0, 255))
        aw = int(np.asarray(a, np.uint8).view("<u4")[0])
        bw = int(np.asarray(c, np.uint8).view("<u4")[0])
        hit, n1, n2 = swar_word(aw, bw, D)
        fin = (a != 255) & (c != 255)
        s = a.astype(np.int64) + c
        assert hit == bool(np.any(s <= D)), it
        assert n2 == sum(1 << i for i in range(4) if fin[i] and s[i] == D + 1), it
        assert n1 == sum(1 << i for i in range(4) if fin[i] and s[i] == D + 2), it
