"""Host model of the chunked merge join of two sorted labels (QUERY of
Section 3.3 as the batched query kernels and the whole-graph kernel run
it): each step loads G hubs of each label into G lanes, every lane finds its
hub of the first chunk in the second chunk by a halving search across the
lanes, and the chunk(s) whose last hub is smaller advance.  Checked against
the minimum over common hubs on random labels of every length mix."""
import numpy as np
import pytest

PAST = 0xFFFFFFFF


def chunked_min(ha, da, hb, db, G):
    best = 255
    ia = ib = 0
    la, lb = len(ha), len(hb)
    while ia < la and ib < lb:
        ca = [ha[ia + g] if ia + g < la else PAST for g in range(G)]
        cb = [hb[ib + g] if ib + g < lb else PAST for g in range(G)]
        for g in range(G):
            lo = 0
            s = G // 2
            while s >= 1:
                if cb[lo + s - 1] < ca[g]:
                    lo += s
                s //= 2
            if cb[lo] == ca[g] and ca[g] != PAST:
                best = min(best, da[ia + g] + db[ib + lo])
        if ca[-1] <= cb[-1]:
            ia += G
        if cb[-1] <= ca[-1]:
            ib += G
    return best


@pytest.mark.parametrize("G", [16, 32, 64])
def test_chunked_merge_join(G):
    rng = np.random.default_rng(G)
    for it in range(600):
        universe = int(rng.integers(1, 400))
        la, lb = (int(x) for x in rng.integers(0, 200, 2))
        ha = np.sort(rng.choice(universe, size=min(la, universe), replace=False))
        hb = np.sort(rng.choice(universe, size=min(lb, universe), replace=False))
        da = rng.integers(0, 120, len(ha))
        db = rng.integers(0, 120, len(hb))
        common = {int(h): int(d) for h, d in zip(ha, da)}
        want = min([common[int(h)] + int(d) for h, d in zip(hb, db) if int(h) in common] + [255])
        got = chunked_min([int(x) for x in ha], [int(x) for x in da],
                          [int(x) for x in hb], [int(x) for x in db], G)
        assert got == want, (it, G)
