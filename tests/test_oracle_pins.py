"""Pins of the CPU oracle against what the paper and the mathematics fix.

- brute force over every reaction subset (Definitions 1-3, exact arithmetic);
- closed forms: Lemma 2's type-I chains with Eq. 3's flux ratios (golden file),
  k parallel routes, 2^k for k diamonds in series, a*b for an AND-join, and the
  number of simple source->sink paths of graph-like networks (networkx);
- invariants of every output (balance, signs, primitivity, minimality);
- metamorphic relations (relabelling, row scaling, a dead end, a duplicated
  reversible column);
- caps: a depth cap filters by support size, a frontier cap returns a subset;
- mutants: source-level mistakes planted in a copy of the oracle must fail a pin.
"""
import json
import os
import shutil
import subprocess

import networkx as nx
import numpy as np
import pytest

import brute
import oracle
from invariants import check_result, keys_to_ints
from paper_1804_02867_amd import netgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TINY_SEEDS = [0, 1, 3, 4, 5, 6]


def _run(net, x, **kw):
    S, rev, ext = net.arrays()
    return oracle.enumerate_pathways(S, rev, ext, x, **kw)


def _as_pairs(res):
    return list(zip(keys_to_ints(res.keys), res.flux.tolist()))


@pytest.fixture(scope="module")
def tiny_circuits():
    cache = {}

    def get(seed):
        if seed not in cache:
            net = netgen.tiny(seed)
            S, rev, ext = net.arrays()
            cache[seed] = brute.circuits(S, ext)
        return cache[seed]
    return get


# ------------------------------------------------------------------ brute force

@pytest.mark.parametrize("seed", TINY_SEEDS)
def test_oracle_equals_brute_force(seed, tiny_circuits):
    net = netgen.tiny(seed)
    S, rev, ext = net.arrays()
    circ = tiny_circuits(seed)
    for x in net.targets:
        expect = brute.elementary_pathways(S, rev, ext, x, circ=circ)
        got = _run(net, x)
        assert got.status == oracle.COMPLETE
        assert _as_pairs(got) == expect
        check_result(S, rev, ext, x, got.keys, got.flux)


def test_brute_force_lift_matches_rationals(tiny_circuits):
    """The mod-p -> integer lift of the brute force agrees with exact rationals."""
    net = netgen.tiny(1)
    S, rev, ext = net.arrays()
    Sint = np.asarray(S, np.int64)[ext == 0]
    for E, cols, v in tiny_circuits(1)[:200]:
        M = [[int(Sint[i, j]) for j in cols] for i in range(Sint.shape[0])]
        basis = brute.nullspace_fraction(M, len(cols))
        assert len(basis) == 1
        ref = brute.primitive(basis[0])
        assert ref == v or ref == [-a for a in v]


def test_depth_cap_filters_by_size(tiny_circuits):
    net = netgen.tiny(0)
    S, rev, ext = net.arrays()
    for x in net.targets:
        full = _as_pairs(_run(net, x))
        for D in (3, 6, 9):
            capped = _run(net, x, depth_cap=D)
            want = [(e, f) for e, f in full if bin(e).count("1") <= D]
            assert _as_pairs(capped) == want
            bigger = any(bin(e).count("1") > D for e, _ in full)
            if bigger:
                assert capped.status & oracle.DEPTH_CAPPED


def test_frontier_cap_gives_subset():
    net = netgen.tiny(0)
    x = net.targets[0]
    full = set(keys_to_ints(_run(net, x).keys))
    for cap in (5, 50, 500):
        r = _run(net, x, frontier_cap=cap)
        assert r.status & oracle.FRONTIER_TRUNCATED
        assert set(keys_to_ints(r.keys)) <= full
        assert (r.levels[:, 5] <= cap).all()


# ----------------------------------------------------------------- closed forms

def test_chain_fluxes_follow_eq3():
    with open(os.path.join(GOLDEN, "chain_eq3.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        for reversible in (False, True):
            net = netgen.chain([tuple(s) for s in case["steps"]], reversible=reversible)
            r = _run(net, net.targets[-1])
            assert r.count == 1
            assert r.flux[0].tolist() == case["flux"]


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_parallel_routes(k):
    net = netgen.parallel_routes(k)
    r = _run(net, net.targets[-1])
    assert r.count == k
    check_result(*net.arrays(), net.targets[-1], r.keys, r.flux)


@pytest.mark.parametrize("k", [1, 2, 4, 6, 8])
def test_diamonds_count_two_to_the_k(k):
    net = netgen.diamonds(k)
    r = _run(net, net.targets[-1])
    assert r.count == 2 ** k
    assert (r.flux[r.flux != 0] == 1).all()


@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (4, 2), (3, 3)])
def test_and_join_counts_multiply(a, b):
    net = netgen.and_join(a, b)
    r = _run(net, net.targets[-1])
    assert r.count == a * b
    check_result(*net.arrays(), net.targets[-1], r.keys, r.flux)


@pytest.mark.parametrize("seed", range(8))
def test_graph_like_counts_simple_paths(seed):
    net = netgen.graph_like(seed, m_int=8, n_edges=16)
    G = nx.DiGraph()
    G.add_nodes_from(range(net.m_int))
    G.add_edges_from(net.meta["edges"])
    expect = sum(1 for _ in nx.all_simple_paths(G, 0, net.m_int - 1))
    r = _run(net, net.targets[-1])
    assert r.count == expect
    check_result(*net.arrays(), net.targets[-1], r.keys, r.flux)


# ------------------------------------------------------------------ metamorphic

def test_relabelling_internal_metabolites():
    net = netgen.tiny(3)
    S, rev, ext = net.arrays()
    rng = np.random.default_rng(7)
    perm = np.r_[rng.permutation(net.m_int), np.arange(net.m_int, net.m)]
    for x in net.targets:
        a = _run(net, x)
        b = oracle.enumerate_pathways(S[perm], rev, ext[perm], int(np.nonzero(perm == x)[0][0]))
        assert _as_pairs(a) == _as_pairs(b)


def test_relabelling_reactions():
    net = netgen.tiny(1)
    S, rev, ext = net.arrays()
    rng = np.random.default_rng(3)
    perm = rng.permutation(net.n)             # new column c holds old column perm[c]
    for x in net.targets:
        a = _run(net, x)
        b = oracle.enumerate_pathways(S[:, perm], rev[perm], ext, x)
        mapped = sorted((sum(1 << int(np.nonzero(perm == j)[0][0]) for j in range(net.n) if (e >> j) & 1),
                         [f[perm[c]] for c in range(net.n)]) for e, f in _as_pairs(a))
        assert _as_pairs(b) == mapped


def test_scaling_an_internal_row():
    net = netgen.tiny(4)
    S, rev, ext = net.arrays()
    for i, c in [(0, 2), (3, -1), (7, 3)]:
        S2 = S.copy()
        S2[i] *= c
        for x in net.targets:
            assert _as_pairs(_run(net, x)) == _as_pairs(oracle.enumerate_pathways(S2, rev, ext, x))


def test_dead_end_reaction_changes_nothing():
    net = netgen.tiny(0)
    S, rev, ext = net.arrays()
    m, n = S.shape
    # new internal metabolite Z (placed last among internal rows is not needed: ext stays)
    S2 = np.zeros((m + 1, n + 1), np.int32)
    S2[:m, :n] = S
    S2[0, n] = -1          # A -> Z, Z consumed by nothing
    S2[m, n] = 1
    ext2 = np.r_[ext, 0].astype(np.uint8)
    rev2 = np.r_[rev, 0].astype(np.uint8)
    for x in net.targets:
        a = _as_pairs(_run(net, x))
        b = oracle.enumerate_pathways(S2, rev2, ext2, x)
        assert [(e, f[:n]) for e, f in _as_pairs(b)] == a


def test_duplicated_reversible_column_doubles_its_pathways():
    net = netgen.tiny(1)
    S, rev, ext = net.arrays()
    r = int(np.nonzero(rev[:net.n_int])[0][0])
    S2 = np.c_[S, S[:, r]]
    rev2 = np.r_[rev, 1].astype(np.uint8)
    for x in net.targets:
        a = _as_pairs(_run(net, x))
        b = oracle.enumerate_pathways(S2, rev2, ext, x)
        through = [(e, f) for e, f in a if (e >> r) & 1]
        assert b.count == len(a) + len(through)
        twins = {(e & ~(1 << r)) | (1 << net.n) for e, _ in through}
        assert twins <= set(keys_to_ints(b.keys))


# ----------------------------------------------------------------------- mutants

MUTANTS = {
    "forward flow ignores reversible consumers": ("ok = N->rev[r] || s < 0;", "ok = s < 0;"),
    "backward flow takes consumers": ("else ok = N->rev[r] || s > 0;", "else ok = N->rev[r] || s < 0;"),
    "closed pathways not extended": ("if (hit) cand[k++] = r;", "(void)hit;"),
    "covered demands three touches": ("(a + b + c >= 2)", "(a + b + c >= 3)"),
    "wrong back-substitution sign": ("v[pc] = (p > 0) ? -(sum / g) : (sum / g);",
                                     "v[pc] = (p > 0) ? (sum / g) : -(sum / g);"),
    "sign feasibility not checked": ("else if (s != sgn) return 0;", "else if (s != sgn) {}"),
    "zero flux entries accepted": ("for (int j = 0; j < k; ++j) if (v[j] == 0) return 0;", ""),
}


def _mutant_lib(tmp_path, name, old, new):
    src = open(oracle._SRC).read()
    assert old in src, name
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", "-o", str(lib), str(path)], check=True)
    return oracle.bind(str(lib))


def _pins_pass(lib, tiny_circuits):
    try:
        for seed in (1, 3):
            net = netgen.tiny(seed)
            S, rev, ext = net.arrays()
            circ = tiny_circuits(seed)
            for x in net.targets:
                got = oracle.enumerate_pathways(S, rev, ext, x, lib=lib)
                if _as_pairs(got) != brute.elementary_pathways(S, rev, ext, x, circ=circ):
                    return False
        for net in (netgen.diamonds(3), netgen.and_join(2, 2), netgen.chain([(2, 3), (3, 1), (1, 2)])):
            S, rev, ext = net.arrays()
            got = oracle.enumerate_pathways(S, rev, ext, net.targets[-1], lib=lib)
            check_result(S, rev, ext, net.targets[-1], got.keys, got.flux)
        return True
    except (AssertionError, RuntimeError):
        return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path, tiny_circuits):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    old, new = MUTANTS[name]
    lib = _mutant_lib(tmp_path, name, old, new)
    assert not _pins_pass(lib, tiny_circuits), f"mutant survived: {name}"


def test_unmutated_oracle_passes_the_same_pins(tiny_circuits):
    assert _pins_pass(oracle._load(), tiny_circuits)
