"""Host model of the prune tests' LDS root table (k_win_test): buckets of
four 32-bit slots holding hub << 8 | distance (or 0xFFFFFFFF when free),
filled in order by linear probing over buckets; a lookup decodes a bucket
with xor and min (slot ^ (h << 8) is the distance exactly when the hub
matches, at least 256 otherwise) and stops at a bucket with a free slot.
Checked against a dictionary on random labels, hubs below 2^24 - 1."""
import numpy as np

EMPTY = 0xFFFFFFFF


def lds_hash(h):
    x = (h & 0xFFFFFF) * 0x9E3779 & 0xFFFFFFFF  # low 32 bits of a 24 x 24 product
    return x ^ (x >> 13)


def build(label, nb):
    tab = [[EMPTY] * 4 for _ in range(nb)]
    for h, d in label.items():
        b = lds_hash(h) & (nb - 1)
        while True:
            free = [i for i in range(4) if tab[b][i] == EMPTY]
            if free:
                tab[b][free[0]] = (h << 8) | d
                break
            b = (b + 1) & (nb - 1)
    return tab


def bucket_dist(q, hk):
    return min(min(q[0] ^ hk, q[1] ^ hk, q[2] ^ hk), q[3] ^ hk, 255)


def lookup(tab, h):
    nb = len(tab)
    b = lds_hash(h) & (nb - 1)
    while True:
        d = bucket_dist(tab[b], h << 8)
        if d != 255 or tab[b][3] == EMPTY:
            return d
        b = (b + 1) & (nb - 1)


def test_lookup_matches_the_label():
    rng = np.random.default_rng(3)
    for it in range(300):
        size = int(rng.integers(1, 1025))
        nb = 4
        while nb < size:
            nb <<= 1
        hubs = rng.choice(2**24 - 1, size=size, replace=False)
        label = {int(h): int(rng.integers(0, 255)) for h in hubs}
        tab = build(label, nb)
        for h, d in list(label.items())[:50]:
            assert lookup(tab, h) == d, it
        others = rng.integers(0, 2**24 - 1, 50)
        for h in others:
            assert lookup(tab, int(h)) == label.get(int(h), 255), it


def test_empty_slot_never_matches():
    # a free slot xor any hub key below 2^24 - 1 stays at 256 or more
    for h in (0, 1, 12345, 2**24 - 2):
        assert (EMPTY ^ (h << 8)) >= 256
