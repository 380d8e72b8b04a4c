"""Seeded synthetic metabolic networks (input data only).

This module builds stoichiometric matrices and nothing else: it holds none of
the traversal's arithmetic, so both the CPU oracle's tests and the GPU path can
draw their inputs from it without sharing any of the method.

A network is S (int32, m x n, rows = metabolites, columns = reactions; S[i,j] > 0
means reaction j produces metabolite i, < 0 consumes it, Section 2.1), the
per-reaction reversibility flags and the per-metabolite external flags.
Layout: internal metabolites first, then external ones; internal reactions
first, then one exchange reaction per external metabolite.  Exchange k is the
reversible reaction u_k <=> x_k with coefficient 1, where u_k is an internal
metabolite and x_k = m_int + k is touched by no other reaction (these are the
paper's boundary reactions, Section 2.1).

Workload shapes (all seeded with numpy's PCG64 default_rng):
  tiny      12 internal metabolites, 16 internal reactions (4 reversible),
            3 exchanges, coefficients {1: .85, 2: .15}            (CHO-core shape)
  central   60 / 90 (20 % reversible) / 10 exchanges, coefficients
            {1: .8, 2: .15, 3: .05}, 5 currency hubs each in 25 % of reactions
  genome    400 / 600 (30 % reversible) / 40 exchanges, power-law metabolite
            degrees (exponent 2.2, degrees 2..120), coefficients as central
  batch     per network i: seed 100000+i, m log-uniform in [10, 80], n log-uniform
            in [15, 120], generator as central
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

COEF_TINY = ((1, 2), (0.85, 0.15))
COEF_CENTRAL = ((1, 2, 3), (0.8, 0.15, 0.05))


def _round_half_up(x: float) -> int:
    return int(math.floor(x + 0.5))


@dataclass
class Network:
    S: np.ndarray            # int32 [m, n]
    rev: np.ndarray          # uint8 [n]
    ext: np.ndarray          # uint8 [m]
    m_int: int
    n_int: int
    name: str = ""
    attempts: int = 1        # rejection-sampling attempts used for connectivity
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.S.shape[0])

    @property
    def n(self) -> int:
        return int(self.S.shape[1])

    @property
    def targets(self) -> list[int]:
        """External metabolites (candidate targets), in index order."""
        return [int(i) for i in np.nonzero(self.ext)[0]]

    def arrays(self):
        return (np.ascontiguousarray(self.S, dtype=np.int32),
                np.ascontiguousarray(self.rev, dtype=np.uint8),
                np.ascontiguousarray(self.ext, dtype=np.uint8))


def _connected(S: np.ndarray) -> bool:
    """Is the bipartite metabolite-reaction graph (all rows) connected?"""
    m, n = S.shape
    parent = list(range(m + n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    rows, cols = np.nonzero(S)
    for i, j in zip(rows.tolist(), cols.tolist()):
        ra, rb = find(i), find(m + j)
        if ra != rb:
            parent[ra] = rb
    root = find(0)
    return all(find(v) == root for v in range(m + n))


def _add_exchanges(rng, S, m_int, n_int, n_ex):
    for k in range(n_ex):
        u = int(rng.integers(0, m_int))
        S[u, n_int + k] = -1
        S[m_int + k, n_int + k] = 1


def _finish(S, m_int, n_int, n_ex, rev_int, name, attempts, meta=None):
    m, n = S.shape
    rev = np.zeros(n, np.uint8)
    rev[rev_int] = 1
    rev[n_int:] = 1
    ext = np.zeros(m, np.uint8)
    ext[m_int:] = 1
    return Network(S.astype(np.int32), rev, ext, m_int, n_int, name, attempts, meta or {})


def uniform_network(rng, m_int, n_int, n_ex, rev_frac=None, n_rev=None, coef=COEF_CENTRAL,
                    n_hub=0, hub_frac=0.25, name="", max_attempts=10000):
    """Internal reactions with 1-3 substrates and 1-3 products drawn uniformly from
    the non-hub metabolites (distinct, sides disjoint), coefficients from `coef`.
    Each hub h < n_hub is then added to exactly round(hub_frac * n_int) reactions as
    a substrate or product (probability 1/2) with a coefficient from `coef`.
    The whole draw is repeated from the same stream until the bipartite graph is
    connected."""
    vals, probs = coef
    pool = np.arange(n_hub, m_int)
    if pool.size < 6:
        raise ValueError("need at least 6 non-hub metabolites")
    if n_rev is None:
        n_rev = _round_half_up(rev_frac * n_int)
    for attempt in range(1, max_attempts + 1):
        S = np.zeros((m_int + n_ex, n_int + n_ex), np.int64)
        for j in range(n_int):
            ns = int(rng.integers(1, 4))
            npr = int(rng.integers(1, 4))
            mets = rng.choice(pool, size=ns + npr, replace=False)
            cf = rng.choice(vals, size=ns + npr, p=probs)
            S[mets[:ns], j] = -cf[:ns]
            S[mets[ns:], j] = cf[ns:]
        n_hub_rx = _round_half_up(hub_frac * n_int)
        for h in range(n_hub):
            rx = rng.choice(n_int, size=n_hub_rx, replace=False)
            side = rng.random(n_hub_rx) < 0.5
            cf = rng.choice(vals, size=n_hub_rx, p=probs)
            S[h, rx] = np.where(side, -cf, cf)
        _add_exchanges(rng, S, m_int, n_int, n_ex)
        rev_int = rng.choice(n_int, size=n_rev, replace=False)
        if _connected(S):
            return _finish(S, m_int, n_int, n_ex, rev_int, name, attempt,
                           {"n_hub": n_hub})
    raise RuntimeError(f"no connected network after {max_attempts} attempts")


def powerlaw_network(rng, m_int, n_int, n_ex, rev_frac, coef=COEF_CENTRAL, exponent=2.2,
                     dmin=2, dmax=120, name="", max_attempts=1000):
    """Chung-Lu style draw: each metabolite gets a weight d_i from the discrete power
    law P(d) ~ d^-exponent on [dmin, dmax]; each reaction picks its 2-6 distinct
    metabolites with probability proportional to d_i.  A metabolite left without
    any reaction replaces a random slot whose metabolite appears at least twice,
    so every metabolite is used.  Repeated until connected."""
    vals, probs = coef
    ks = np.arange(dmin, dmax + 1, dtype=np.float64)
    pk = ks ** (-exponent)
    pk /= pk.sum()
    n_rev = _round_half_up(rev_frac * n_int)
    for attempt in range(1, max_attempts + 1):
        d = rng.choice(ks, size=m_int, p=pk)
        w = d / d.sum()
        slots = []                       # per reaction: (mets, n_sub)
        for j in range(n_int):
            ns = int(rng.integers(1, 4))
            npr = int(rng.integers(1, 4))
            mets = rng.choice(m_int, size=ns + npr, replace=False, p=w)
            slots.append([mets, ns])
        count = np.zeros(m_int, np.int64)
        for mets, _ in slots:
            count[mets] += 1
        for i in np.nonzero(count == 0)[0].tolist():
            for _ in range(100000):
                j = int(rng.integers(0, n_int))
                mets = slots[j][0]
                p = int(rng.integers(0, mets.size))
                if count[mets[p]] >= 2 and i not in mets:
                    count[mets[p]] -= 1
                    mets[p] = i
                    count[i] += 1
                    break
        S = np.zeros((m_int + n_ex, n_int + n_ex), np.int64)
        for j, (mets, ns) in enumerate(slots):
            cf = rng.choice(vals, size=mets.size, p=probs)
            S[mets[:ns], j] = -cf[:ns]
            S[mets[ns:], j] = cf[ns:]
        _add_exchanges(rng, S, m_int, n_int, n_ex)
        rev_int = rng.choice(n_int, size=n_rev, replace=False)
        if _connected(S):
            return _finish(S, m_int, n_int, n_ex, rev_int, name, attempt,
                           {"exponent": exponent, "dmin": dmin, "dmax": dmax})
    raise RuntimeError(f"no connected network after {max_attempts} attempts")


# ---------------------------------------------------------------- workload shapes

def tiny(seed: int) -> Network:
    rng = np.random.default_rng(seed)
    return uniform_network(rng, 12, 16, 3, n_rev=4, coef=COEF_TINY, name=f"tiny/{seed}")


def central(seed: int) -> Network:
    rng = np.random.default_rng(seed)
    return uniform_network(rng, 60, 90, 10, rev_frac=0.2, coef=COEF_CENTRAL, n_hub=5,
                           name=f"central/{seed}")


def genome(seed: int) -> Network:
    rng = np.random.default_rng(seed)
    return powerlaw_network(rng, 400, 600, 40, rev_frac=0.3, name=f"genome/{seed}")


def batch_member(i: int) -> Network:
    """Batch network i (seed 100000 + i): m_int log-uniform in [10, 80] and n_int
    log-uniform in [15, 120], drawn independently, then the central-shape
    generator.  A size pair whose networks fail to connect within 200 draws, or
    with too few reaction slots to touch every metabolite (3 n < m), is replaced
    by the next pair from the same stream."""
    rng = np.random.default_rng(100000 + i)
    while True:
        m = _round_half_up(math.exp(rng.uniform(math.log(10), math.log(80))))
        n = _round_half_up(math.exp(rng.uniform(math.log(15), math.log(120))))
        if 3 * n < m:
            continue
        n_ex = max(2, _round_half_up(m / 6))
        n_hub = 5 if m >= 30 else max(1, m // 6)
        try:
            return uniform_network(rng, m, n, n_ex, rev_frac=0.2, coef=COEF_CENTRAL, n_hub=n_hub,
                                   name=f"batch/{i}", max_attempts=200)
        except RuntimeError:
            continue


SHAPES = {"tiny": tiny, "central": central, "genome": genome}


# ------------------------------------------------------ hand-built closed forms
# Small structured networks whose pathway counts are known in closed form
# (Lemma 2's chains, parallel routes, diamonds, AND-joins).  Input data only.

def _net_from_columns(m_int, cols, rev_flags, n_ext_rows, name):
    """cols: list of dicts {row: coef}; rows >= m_int are external."""
    m = m_int + n_ext_rows
    n = len(cols)
    S = np.zeros((m, n), np.int32)
    for j, col in enumerate(cols):
        for i, c in col.items():
            S[i, j] = c
    rev = np.array(rev_flags, np.uint8)
    ext = np.zeros(m, np.uint8)
    ext[m_int:] = 1
    return Network(S, rev, ext, m_int, n, name)


def chain(coefs: list[tuple[int, int]], reversible=False) -> Network:
    """x_in -> A_0 ; c0 A_0 -> d0 A_1 ; ... ; A_last -> x_out.
    coefs[k] = (c, d) for the k-th internal step; len(coefs)+1 internal metabolites.
    External rows: x_in = m_int, x_out = m_int + 1 (the target)."""
    L = len(coefs)
    m_int = L + 1
    xin, xout = m_int, m_int + 1
    cols = [{xin: -1, 0: 1}]
    for k, (c, d) in enumerate(coefs):
        cols.append({k: -c, k + 1: d})
    cols.append({L: -1, xout: 1})
    return _net_from_columns(m_int, cols, [int(reversible)] * len(cols), 2, "chain")


def parallel_routes(k: int) -> Network:
    """x_in -> A, k routes A -> B (each via its own intermediate), B -> x_out."""
    # metabolites: A=0, B=1, I_j = 2+j ; externals x_in, x_out
    m_int = 2 + k
    xin, xout = m_int, m_int + 1
    cols = [{xin: -1, 0: 1}]
    for j in range(k):
        cols.append({0: -1, 2 + j: 1})
        cols.append({2 + j: -1, 1: 1})
    cols.append({1: -1, xout: 1})
    return _net_from_columns(m_int, cols, [0] * len(cols), 2, f"routes{k}")


def diamonds(k: int) -> Network:
    """k diamonds in series: N_0 -> (U_j | L_j) -> N_{j+1}; 2^k routes in total."""
    # metabolites: N_0..N_k = 0..k, then U_j = k+1+2j, L_j = k+2+2j
    m_int = (k + 1) + 2 * k
    xin, xout = m_int, m_int + 1
    cols = [{xin: -1, 0: 1}]
    for j in range(k):
        u, l = k + 1 + 2 * j, k + 2 + 2 * j
        cols.append({j: -1, u: 1})
        cols.append({u: -1, j + 1: 1})
        cols.append({j: -1, l: 1})
        cols.append({l: -1, j + 1: 1})
    cols.append({k: -1, xout: 1})
    return _net_from_columns(m_int, cols, [0] * len(cols), 2, f"diamonds{k}")


def and_join(a: int, b: int) -> Network:
    """Two independent supplies joined by one AND reaction P + Q -> Z -> x_out.
    P has `a` parallel routes from x_in, Q has `b`: a*b pathways."""
    # metabolites: S_in=0, P=1, Q=2, Z=3, then route intermediates
    m_int = 4 + a + b
    xin, xout = m_int, m_int + 1
    cols = [{xin: -2, 0: 2}]                   # x_in -> S_in (coefficient 2 on both sides)
    for j in range(a):
        cols.append({0: -1, 4 + j: 1})
        cols.append({4 + j: -1, 1: 1})
    for j in range(b):
        cols.append({0: -1, 4 + a + j: 1})
        cols.append({4 + a + j: -1, 2: 1})
    cols.append({1: -1, 2: -1, 3: 1})
    cols.append({3: -1, xout: 1})
    return _net_from_columns(m_int, cols, [0] * len(cols), 2, f"andjoin{a}x{b}")


def graph_like(seed: int, m_int: int = 8, n_edges: int = 14, rev_p: float = 0.0) -> Network:
    """Every internal reaction is a 1 -> 1 edge with coefficient 1 between internal
    metabolites (a digraph); x_in feeds metabolite 0 and metabolite m_int-1 drains
    to x_out.  Irreversible, so source->target pathways are the simple directed
    paths from 0 to m_int-1 plus the directed cycles that the target pathway
    cannot touch (those do not produce the target and are not counted)."""
    rng = np.random.default_rng(seed)
    xin, xout = m_int, m_int + 1
    edges = set()
    while len(edges) < n_edges:
        u, v = (int(x) for x in rng.choice(m_int, 2, replace=False))
        edges.add((u, v))
    edges = sorted(edges)
    cols = [{xin: -1, 0: 1}]
    for (u, v) in edges:
        cols.append({u: -1, v: 1})
    cols.append({m_int - 1: -1, xout: 1})
    net = _net_from_columns(m_int, cols, [0] * len(cols), 2, f"graph{seed}")
    net.meta["edges"] = edges
    return net


def learn_member(seed: int) -> Network:
    """Network of the learned-ordering workload: the genome-scale generator
    (power-law metabolite degrees, 30% reversible) at a tenth of its size, 40
    internal metabolites, 60 reactions and 4 exchanges, small enough for the plain
    traversal to finish exhaustively at depth cap 16."""
    rng = np.random.default_rng(seed)
    return powerlaw_network(rng, 40, 60, 4, 0.3, name=f"learn/{seed}")
