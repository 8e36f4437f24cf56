"""SHA-256 digests of an exported index, for comparing large indexes with
stored oracle results without keeping the oracle's arrays.

The export layout is the one both sides produce (vertices in rank order,
``off int64[n+1]``, ``hub uint32``, ``dist uint8``, no sentinels,
``bp_d uint8[n][t]``, ``bp_m1``/``bp_0 uint64[n][t]``); every array is hashed
little-endian.  Besides one digest per array and one over all of them in
that order, the vertices are cut into blocks of ``BLOCK`` ranks and each block
gets a short digest, so a mismatch names the ranks where it sits.
"""
from __future__ import annotations

import hashlib

import numpy as np

BLOCK = 1 << 14
ARRAYS = ("off", "hub", "dist", "bp_d", "bp_m1", "bp_0")


def _le(a, dt):
    return np.ascontiguousarray(a, dtype=np.dtype(dt).newbyteorder("<"))


def index_digests(off, hub, dist, bp_d, bp_m1, bp_0, block: int = BLOCK) -> dict:
    arrs = {"off": _le(off, "i8"), "hub": _le(hub, "u4"), "dist": _le(dist, "u1"),
            "bp_d": _le(bp_d, "u1"), "bp_m1": _le(bp_m1, "u8"), "bp_0": _le(bp_0, "u8")}
    n = len(arrs["off"]) - 1
    out = {"n": int(n), "entries": int(arrs["off"][-1]) if n >= 0 else 0}
    every = hashlib.sha256()
    for k in ARRAYS:
        h = hashlib.sha256(memoryview(arrs[k]).cast("B"))
        every.update(memoryview(arrs[k]).cast("B"))
        out[k] = h.hexdigest()
    out["all"] = every.hexdigest()
    o = arrs["off"]
    bd = arrs["bp_d"].reshape(n, -1) if n else arrs["bp_d"]
    b1 = arrs["bp_m1"].reshape(n, -1) if n else arrs["bp_m1"]
    b0 = arrs["bp_0"].reshape(n, -1) if n else arrs["bp_0"]
    blocks = []
    for v0 in range(0, n, block):
        v1 = min(n, v0 + block)
        a, b = int(o[v0]), int(o[v1])
        h = hashlib.sha256()
        h.update(memoryview(np.ascontiguousarray(np.diff(o[v0:v1 + 1]))).cast("B"))
        h.update(memoryview(arrs["hub"][a:b]).cast("B"))
        h.update(memoryview(arrs["dist"][a:b]).cast("B"))
        for part in (bd, b1, b0):
            h.update(memoryview(np.ascontiguousarray(part[v0:v1])).cast("B"))
        blocks.append(h.hexdigest()[:16])
    out["blocks"] = blocks
    out["block"] = int(block)
    return out


def answers_digest(ans) -> dict:
    a = np.ascontiguousarray(ans)
    hist = np.bincount(a.astype(np.int64).ravel(), minlength=256) if a.dtype == np.uint8 else None
    d = {"count": int(a.size), "sha256": hashlib.sha256(memoryview(a).cast("B")).hexdigest()}
    if hist is not None:
        d["hist"] = {str(i): int(c) for i, c in enumerate(hist) if c}
    return d


def compare(got: dict, want: dict) -> list[str]:
    """Human-readable differences between two index_digests() results."""
    bad = []
    for k in ("n", "entries") + ARRAYS + ("all",):
        if got.get(k) != want.get(k):
            bad.append(f"{k}: {got.get(k)} != {want.get(k)}")
    if got.get("blocks") != want.get("blocks"):
        B = want.get("block", BLOCK)
        diff = [i for i, (x, y) in enumerate(zip(got.get("blocks", []), want.get("blocks", [])))
                if x != y]
        bad.append(f"{len(diff)} vertex blocks differ, first ranks "
                   f"{[i * B for i in diff[:8]]}")
    return bad
