"""The genome-shaped workload at its full caps (400 internal metabolites, 600 + 40
reactions, depth cap 40, frontier cap 2^26, room for 2^30 distinct children per
level): counters of the levels the oracle can enumerate agree exactly, every level
respects the cap, the status flags are set, and any pathway found is elementary."""
import time

import numpy as np
import pytest

import oracle
from invariants import check_result
from paper_1804_02867_amd import netgen

pytestmark = pytest.mark.gpu

efm = pytest.importorskip("paper_1804_02867_amd.efm")


def test_genome_at_full_caps():
    net = netgen.genome(0)
    x = net.targets[0]
    S, rev, ext = net.arrays()
    g = efm.Network(S, rev, ext)
    cap = 1 << 26
    print("case genome/0 depth cap 40 frontier cap 2^26", flush=True)
    t = time.perf_counter()
    r = efm.enumerate_pathways(g, x, depth_cap=40, frontier_cap=cap, unique_cap=1 << 30, found_cap=1 << 16)
    dt = time.perf_counter() - t
    kept = [lv["kept"] for lv in r.levels]
    print(f"genome full caps: {len(r.levels)} levels, peak frontier {max(kept)}, "
          f"{sum(lv['parents'] for lv in r.levels)} parents, {r.count} pathways, {dt:.1f} s", flush=True)
    assert len(r.levels) == 40
    assert r.status & efm.FRONTIER_TRUNCATED and r.status & efm.DEPTH_CAPPED
    assert all(k <= cap for k in kept) and max(kept) == cap
    # the first levels stay far below the cap: the oracle enumerates them exactly
    want = oracle.enumerate_pathways(S, rev, ext, x, depth_cap=5)
    for i in range(4):
        got = [r.levels[i][f] for f in ("children", "unique", "independent", "emitted", "kept")]
        assert got == want.levels[i, 1:].tolist(), i
        if i > 0:                            # level 1's parent is the empty pathway on the GPU
            assert r.levels[i]["parents"] == want.levels[i, 0], i
    if r.count:
        check_result(S, rev, ext, x, r.keys, r.flux, 40)
