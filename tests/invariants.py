"""Properties every result must have, whatever produced it (Definitions 2-3).

All checks use Python integers (exact)."""
from __future__ import annotations

from math import gcd

import numpy as np


def keys_to_ints(keys: np.ndarray) -> list[int]:
    out = []
    for row in np.asarray(keys, dtype=np.uint64):
        v = 0
        for w, word in enumerate(row.tolist()):
            v |= int(word) << (64 * w)
        out.append(v)
    return out


def check_result(S, rev, ext, target, keys, flux, depth_cap=0):
    S = np.asarray(S, dtype=np.int64)
    m, n = S.shape
    internal = [i for i in range(m) if not ext[i]]
    ints = keys_to_ints(keys)
    assert ints == sorted(ints), "not in canonical order"
    assert len(set(ints)) == len(ints), "duplicate pathways"
    supports = []
    for E, v in zip(ints, np.asarray(flux).tolist()):
        v = [int(x) for x in v]
        supp = sum(1 << j for j in range(n) if v[j] != 0)
        assert supp == E, "bitset differs from the flux support"
        if depth_cap > 0:
            assert bin(E).count("1") <= depth_cap
        for i in internal:                                   # S_int v = 0 (Definition 2)
            assert sum(int(S[i, j]) * v[j] for j in range(n)) == 0, "not balanced"
        for j in range(n):                                   # v_irr >= 0 (Definition 2)
            if not rev[j] and v[j] != 0:
                assert v[j] > 0, "irreversible reaction runs backwards"
        assert sum(int(S[target, j]) * v[j] for j in range(n)) > 0, "target not produced"
        g = 0
        for x in v:
            g = gcd(g, abs(x))
        assert g == 1, "flux vector not primitive"
        supports.append(E)
    # minimality (Definition 3): no output's support contains another's
    by_size = sorted(supports, key=lambda e: bin(e).count("1"))
    for a_i, a in enumerate(by_size):
        for b in by_size[a_i + 1:]:
            assert (a & b) != a, "a support contains another"
    return len(ints)
