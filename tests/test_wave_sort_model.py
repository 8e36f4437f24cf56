"""Host model of the root scatter's wave step (k_root_scatter): 64 lanes
sort their (root, lane) keys with a bitonic network of xor partners, the
first lane of each root's run reserves the run's places with one atomic, and
every entry lands at its root's offset plus its rank in the run.  Checked on
random waves: each root's entries get places 0, 1, ... in their original
lane order, and no place is used twice."""
import numpy as np

W = 64
INVALID = 2**31 - 1


def wave_scatter(slots, nvalid, fill):
    """Places (root, index in the root's run) of the wave's valid lanes,
    given the roots' run counters `fill` (updated as the atomics would)."""
    key = [(slots[l] << 6) | l if l < nvalid else INVALID for l in range(W)]
    k = 2
    while k <= W:
        s = k >> 1
        while s > 0:
            other = [key[l ^ s] for l in range(W)]
            key = [min(other[l], key[l]) if ((l & s) == 0) == ((l & k) == 0)
                   else max(other[l], key[l]) for l in range(W)]
            s >>= 1
        k <<= 1
    real = [x != INVALID for x in key]
    root = [x >> 6 for x in key]
    src = [x & 63 for x in key]
    first = [real[l] and (l == 0 or root[l - 1] != root[l]) for l in range(W)]
    starts = sum(1 << l for l in range(W) if first[l])
    nreal = sum(real)
    base = [0] * W
    for l in range(W):  # the leaders' atomics (all at once on the device)
        if first[l]:
            after = starts & ~((2 << l) - 1)
            end = min(nreal, (after & -after).bit_length() - 1 if after else W)
            base[l] = fill.get(root[l], 0)
            fill[root[l]] = base[l] + end - l
    places = {}
    for l in range(W):
        if real[l]:
            r0 = (starts & ((2 << l) - 1)).bit_length() - 1
            places[src[l]] = (root[l], base[r0] + l - r0)
    return key, places


def test_wave_sort_and_runs():
    rng = np.random.default_rng(7)
    for it in range(3000):
        nvalid = int(rng.integers(0, W + 1))
        roots = int(rng.choice([1, 2, 3, 5, 17, 16384]))
        slots = [int(x) for x in rng.integers(0, roots, W)]
        fill = {}
        key, places = wave_scatter(slots, nvalid, fill)
        assert key == sorted(key)
        assert len(set(places.values())) == len(places) == nvalid
        for r in set(slots[:nvalid]):
            lanes = [l for l in range(nvalid) if slots[l] == r]
            assert [places[l] for l in lanes] == [(r, i) for i in range(len(lanes))], it
            assert fill[r] == len(lanes)


def test_waves_continue_a_root_run():
    # a second wave of the same root continues where the first one ended
    fill = {}
    wave_scatter([4] * W, 10, fill)
    _, places = wave_scatter([4] * W, 3, fill)
    assert sorted(places.values()) == [(4, 10), (4, 11), (4, 12)] and fill[4] == 13
