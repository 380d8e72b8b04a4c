"""Learned frontier ordering on the GPU versus the fp64 oracle (oracle/learned.py):
model inputs and trace labels bit-exact, logits and gradients within a bound
derived from the kernels' arithmetic (bf16 operands, fp32 accumulation), one
Adam step, and the learned traversal's invariants."""
import numpy as np
import pytest

import oracle
from invariants import check_result
from oracle import learned as L
from paper_1804_02867_amd import netgen

pytestmark = pytest.mark.gpu

efm = pytest.importorskip("paper_1804_02867_amd.efm")

IN_BITS, IN_COUNTS = 64, 40
F = IN_BITS + 2 * IN_COUNTS
H = 256
U_BF = 2.0 ** -8     # bf16 round-to-nearest relative error (2^-9), doubled
GAM = 2.0 ** -14     # fp32 accumulation of up to ~1000 terms


def bf16_exact(a):
    """Values representable in bf16 (low mantissa bits cleared)."""
    a = np.asarray(a, np.float32)
    return (a.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)


def bf16_rne(a):
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def random_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    P = {"W1": bf16_exact(rng.uniform(-0.5, 0.5, (F, H)) * scale),
         "b1": rng.uniform(-0.2, 0.2, H).astype(np.float32),
         "W2": bf16_exact(rng.uniform(-0.15, 0.15, (H, H)) * scale),
         "b2": rng.uniform(-0.1, 0.1, H).astype(np.float32),
         "w3": bf16_exact(rng.uniform(-0.2, 0.2, H) * scale),
         "b3": np.array([0.1], np.float32)}
    return {k: v.astype(np.float64) for k, v in P.items()}


def random_records(seed, count):
    rng = np.random.default_rng(seed)
    recs = []
    for _ in range(count):
        nb = int(rng.integers(1, 17))
        nc = int(rng.integers(0, 12))
        bits = sorted(rng.choice(IN_BITS, nb, replace=False).tolist())
        mets = sorted(rng.choice(IN_COUNTS, nc, replace=False).tolist())
        codes = rng.integers(1, 8, nc)
        signs = rng.integers(0, 2, nc)
        recs.append([(b, 0) for b in bits] +
                    [(IN_BITS + 2 * m + int(sg), int(c)) for m, c, sg in zip(mets, codes, signs)])
    return recs


def pack(recs):
    ent = np.zeros((len(recs), efm.FEAT_MAX), np.uint16)
    ln = np.zeros(len(recs), np.uint16)
    for i, r in enumerate(recs):
        ent[i, :len(r)] = L.encode(r)
        ln[i] = len(r)
    return ent, ln


def fwd_bounds(P, X):
    """Oracle forward plus per-value bounds on the kernels' deviation from it, and
    the units whose pre-activation lies within that deviation of the kink."""
    f = L.forward(P, X)
    e_z1 = GAM * (np.abs(X) @ np.abs(P["W1"]) + np.abs(P["b1"]))
    e_a1 = U_BF * f["a1"] + e_z1
    e_z2 = e_a1 @ np.abs(P["W2"]) + GAM * (f["a1"] @ np.abs(P["W2"]) + np.abs(P["b2"]))
    e_s = e_z2 @ np.abs(P["w3"]) + GAM * (f["a2"] @ np.abs(P["w3"]) + abs(P["b3"][0]))
    f["amb1"] = np.abs(f["z1"]) <= 2 * e_z1
    f["amb2"] = np.abs(f["z2"]) <= 2 * e_z2
    return f, e_a1, e_z2, e_s, None


def grad_bounds(P, X, y, pw, f, e_a1, e_z2, e_s):
    """Bounds on the gradient kernels' deviation from the oracle.  At a unit whose
    pre-activation is within its error bound of 0 the kernel may take either side
    of the rectifier, so the whole backpropagated term is allowed there."""
    B = X.shape[0]
    s = f["s"]
    sig = 1.0 / (1.0 + np.exp(-s))
    g = (pw * y * (sig - 1.0) + (1.0 - y) * sig) / B
    wmax = np.where(y > 0, pw, 1.0)
    e_g = wmax * (0.25 * e_s + 1e-6) / B
    m1, m2 = f["z1"] > 0, f["z2"] > 0
    a1m, a2m = m1 | f["amb1"], m2 | f["amb2"]
    aw3 = np.abs(P["w3"])
    dz2 = np.outer(g, P["w3"]) * m2
    e_dz2 = np.outer(e_g, aw3) * a2m + np.outer(np.abs(g), aw3) * f["amb2"]
    e_dz2b = e_dz2 + U_BF * (np.abs(dz2) + e_dz2)
    e_a2 = e_z2 * a2m
    adz1 = (np.abs(dz2) @ np.abs(P["W2"]).T)
    e_dz1 = (e_dz2b @ np.abs(P["W2"]).T + GAM * adz1) * a1m + adz1 * f["amb1"]
    adz1 = adz1 * m1
    E = {"b3": np.array([e_g.sum() + GAM * np.abs(g).sum()]),
         "w3": e_g @ (f["a2"] + e_a2) + np.abs(g) @ e_a2 + GAM * (np.abs(g) @ f["a2"]),
         "b2": e_dz2.sum(0) + GAM * np.abs(dz2).sum(0),
         "W2": e_a1.T @ (np.abs(dz2) + e_dz2b) + f["a1"].T @ e_dz2b + GAM * (f["a1"].T @ np.abs(dz2)),
         "W1": np.abs(X).T @ e_dz1 + GAM * (np.abs(X).T @ adz1),
         "b1": e_dz1.sum(0) + GAM * adz1.sum(0)}
    loss_e = float((wmax * e_s).sum() / B) + 1e-6
    return E, loss_e


def model_with(P):
    m = efm.Model(IN_BITS, IN_COUNTS, seed=1)
    m.set_params(L.flatten(P).astype(np.float32))
    return m


def test_record_logits_match_oracle():
    P = random_params(0)
    recs = random_records(1, 300)
    X = L.dense(recs, F)
    f, _, _, e_s, _ = fwd_bounds(P, X)
    print(f"case learned logits records={len(recs)}", flush=True)
    m = model_with(P)
    tr = efm.Traces(IN_BITS, IN_COUNTS, capacity=1024)
    ent, ln = pack(recs)
    tr.append(ent, ln, np.zeros(len(recs), np.uint8))
    got = m.score(tr)
    assert np.all(np.abs(got - f["s"]) <= 2 * e_s + 1e-6), np.max(np.abs(got - f["s"]) - 2 * e_s)
    # a different part of the range and a tail that is not a multiple of the tile
    got2 = m.score(tr, 17, 35)
    assert np.array_equal(got2, got[17:52])


def test_params_roundtrip_and_bf16_copies(tmp_path):
    rng = np.random.default_rng(5)
    m = efm.Model(IN_BITS, IN_COUNTS, seed=3)
    p = m.get_params()
    assert p.size == F * H + H + H * H + H + H + 1
    # non-bf16 master values: the kernels use their round-to-nearest-even copies
    q = (rng.uniform(-0.3, 0.3, p.size)).astype(np.float32)
    m.set_params(q)
    assert np.array_equal(m.get_params(), q)
    recs = random_records(6, 64)
    tr = efm.Traces(IN_BITS, IN_COUNTS, capacity=64)
    ent, ln = pack(recs)
    tr.append(ent, ln, np.zeros(64, np.uint8))
    P = L.unflatten(q.astype(np.float64), F, H)
    for k in ("W1", "W2", "w3"):
        P[k] = bf16_rne(P[k].astype(np.float32)).astype(np.float64)
    f, _, _, e_s, _ = fwd_bounds(P, L.dense(recs, F))
    got = m.score(tr)
    assert np.all(np.abs(got - f["s"]) <= 2 * e_s + 1e-6)
    path = str(tmp_path / "m.bin")
    m.save(path)
    m2 = efm.Model.load(path)
    assert np.array_equal(m2.get_params(), q)
    assert np.array_equal(m2.score(tr), got)


@pytest.mark.parametrize("pw,active", [(1.0, False), (5.0, False), (2.0, True)])
def test_gradient_matches_oracle(pw, active):
    P = random_params(10)
    if active:
        # every rectifier well inside its linear part: no branch is in doubt and
        # the bound is tight
        P["b1"] = P["b1"] + 8.0
        P["b2"] = P["b2"] + 80.0
        P["w3"] = bf16_exact(P["w3"] * 0.01).astype(np.float64)
    recs = random_records(11, 500)
    X = L.dense(recs, F)
    y = (np.random.default_rng(12).random(len(recs)) < 0.3).astype(np.float64)
    f, e_a1, e_z2, e_s, _ = fwd_bounds(P, X)
    if active:
        assert not f["amb1"].any() and not f["amb2"].any() and (f["z1"] > 0).all() and (f["z2"] > 0).all()
    loss, G, _ = L.loss_and_grad(P, X, y, pw)
    E, loss_e = grad_bounds(P, X, y, pw, f, e_a1, e_z2, e_s)
    print(f"case learned grad pw={pw} active={active} items={len(recs)}", flush=True)
    m = model_with(P)
    tr = efm.Traces(IN_BITS, IN_COUNTS, capacity=1024)
    ent, ln = pack(recs)
    tr.append(ent, ln, y.astype(np.uint8))
    gl, gg = m.grad(tr, pos_weight=pw)
    assert abs(gl - loss) <= loss_e
    Gg = L.unflatten(gg.astype(np.float64), F, H)
    for k in L.PARAM_ORDER:
        # rigorous: every entry within the propagated rounding bound
        tol = 2 * E[k] + 1e-9 + 2.0 ** -22 * np.abs(G[k])
        bad = np.abs(Gg[k] - G[k]) > tol
        assert not bad.any(), (k, np.argwhere(bad)[:5], (np.abs(Gg[k] - G[k]) - tol).max())
        # discriminating: the whole block agrees to about the bf16 unit (a
        # misplaced row, column or sign would be off by order one)
        # (units near a kink may flip, so the mixed case allows more)
        rel = np.linalg.norm(Gg[k] - G[k]) / max(np.linalg.norm(G[k]), 1e-30)
        assert rel < (1e-2 if active else 5e-2), (k, rel)
    # rows of inputs absent from the batch get exactly zero gradient
    absent = np.abs(X).sum(0) == 0
    assert np.all(Gg["W1"][absent] == 0)
    # the model is unchanged by a gradient evaluation
    assert np.array_equal(m.get_params(), L.flatten(P).astype(np.float32))


def test_one_adam_step_matches_oracle():
    P = random_params(20)
    recs = random_records(21, 400)
    X = L.dense(recs, F)
    y = (np.random.default_rng(22).random(len(recs)) < 0.5).astype(np.float64)
    _, G, _ = L.loss_and_grad(P, X, y, 2.0)
    M0 = {k: np.zeros_like(v) for k, v in P.items()}
    lr, eps = 1e-3, 1e-8
    P1, _, _ = L.adam_step(P, G, M0, dict(M0), 1, lr, 0.9, 0.999, eps)
    m = model_with(P)
    tr = efm.Traces(IN_BITS, IN_COUNTS, capacity=1024)
    ent, ln = pack(recs)
    tr.append(ent, ln, y.astype(np.uint8))
    print("case learned adam", flush=True)
    st = m.train(tr, epochs=1, batch=len(recs), lr=lr, pos_weight=2.0, eps=eps, seed=0)
    assert st["steps"] == 1
    Q = L.unflatten(m.get_params().astype(np.float64), F, H)
    n_sure = 0
    for k in L.PARAM_ORDER:
        # inputs absent from the batch: zero gradient, so exactly no update
        zero = G[k] == 0
        assert np.array_equal(Q[k][zero], P[k][zero].astype(np.float32).astype(np.float64)), k
        # a first Adam step moves every weight by at most lr
        assert np.all(np.abs(Q[k] - P[k]) <= lr * (1 + 1e-5) + 2.0 ** -22 * np.abs(P[k])), k
        # where the gradient is well above the kernels' gradient error (a few
        # percent of the block's RMS, from the gradient test) its sign is certain,
        # and the step is -lr * g / (|g| + eps)
        rms = np.sqrt(np.mean(G[k] ** 2))
        sure = np.abs(G[k]) > max(0.5 * rms, 1e-6)
        n_sure += int(sure.sum())
        tol = lr * (4 * eps / np.maximum(np.abs(G[k]), 1e-30) + 1e-5) + 2.0 ** -22 * np.abs(P[k])
        diff = np.abs(Q[k] - P1[k])
        assert np.all(diff[sure] <= tol[sure]), (k, (diff - tol)[sure].max())
    assert n_sure > 10000


def test_training_separates_a_planted_rule():
    # label = 1 iff input row 3 is present: a few epochs must separate the classes
    rng = np.random.default_rng(30)
    recs = random_records(31, 4000)
    y = np.array([any(r == 3 and c == 0 for r, c in rec) for rec in recs], np.uint8)
    tr = efm.Traces(IN_BITS, IN_COUNTS, capacity=4096)
    ent, ln = pack(recs)
    tr.append(ent, ln, y)
    m = efm.Model(IN_BITS, IN_COUNTS, seed=4)
    st = m.train(tr, epochs=6, batch=256, lr=2e-3, seed=1)
    assert st["loss_last"] < 0.5 * st["loss_first"]
    s = m.score(tr)
    acc = np.mean((s > 0) == (y > 0))
    assert acc > 0.97, acc
    del rng


def _plain(net, x, D, cap=0):
    g = efm.Network(*net.arrays())
    return g, efm.enumerate_pathways(g, x, depth_cap=D, frontier_cap=cap, unique_cap=1 << 25)


def _tiny_cases():
    for seed in range(6):
        net = netgen.tiny(seed)
        for x in net.targets:
            yield net, x


def test_trace_records_match_oracle_features_and_labels():
    tr = efm.Traces(1024, 400, capacity=1 << 20)
    rng = np.random.default_rng(0)
    n_checked = 0
    for net, x in _tiny_cases():
        S, rev, ext = net.arrays()
        g = efm.Network(S, rev, ext)
        want = oracle.enumerate_pathways(S, rev, ext, x)
        first = len(tr)
        print(f"case learned trace {net.name} x={x}", flush=True)
        info = tr.collect(g, x, neg_per_pos=1.0, neg_min=4, seed=9)
        assert info["pathways"] == want.count
        if info["recorded"] == 0:
            continue
        ent, ln, lab, keys = tr.fetch(first, info["recorded"])
        assert int(lab.sum()) == info["positives"]       # every positive state is kept
        rpos, mpos = L.relabel(S, rev, ext, x)
        pick = rng.choice(len(ln), min(300, len(ln)), replace=False)
        exp_lab = L.label(keys[pick, :1], want.keys) if want.count else np.zeros(len(pick), np.uint8)
        assert np.array_equal(lab[pick], exp_lab)
        for i in pick:
            rs = L.keys_to_reactions(keys[i])
            assert 1 <= len(rs)              # the first frontier holds the target's roots
            feat = L.encode(L.features(S, ext, rs, rpos, mpos, 1024))
            assert np.array_equal(ent[i, :ln[i]], feat), (net.name, x, i)
            n_checked += 1
    assert n_checked > 1000


def test_score_keys_match_oracle():
    net = netgen.learn_member(300001)
    x = net.targets[0]
    S, rev, ext = net.arrays()
    rng = np.random.default_rng(40)
    P = random_params(41)
    Pn = {k: v for k, v in P.items()}
    # widen W1 to the 1024 + 400 inputs the network needs
    big = np.zeros((1024 + 800, H))
    big[:IN_BITS] = P["W1"][:IN_BITS]
    big[1024:1024 + 2 * IN_COUNTS] = P["W1"][IN_BITS:]
    big[IN_BITS:1024] = bf16_exact(rng.uniform(-0.5, 0.5, (1024 - IN_BITS, H)))
    Pn["W1"] = big
    m = efm.Model(1024, 400, seed=2)
    m.set_params(L.flatten(Pn).astype(np.float32))
    g = efm.Network(S, rev, ext)
    keys = np.zeros((200, 1), np.uint64)
    for i in range(200):
        rs = rng.choice(net.n, int(rng.integers(1, 17)), replace=False)
        for r in rs:
            keys[i, 0] |= np.uint64(1) << np.uint64(int(r))
    rpos, mpos = L.relabel(S, rev, ext, x)
    X = L.dense([L.features(S, ext, L.keys_to_reactions(k), rpos, mpos, 1024) for k in keys], 1824)
    f, _, _, e_s, _ = fwd_bounds(Pn, X)
    got = m.score_keys(g, x, keys)
    assert np.all(np.abs(got - f["s"]) <= 2 * e_s + 1e-6)


def test_learned_traversal_reduces_to_plain_on_tiny_networks():
    # budget above every level: the oracle's exhaustive set; a constant score (all
    # weights zero): the oracle's canonical truncation at the same budget
    m = efm.Model(1024, 400, seed=7)
    zero = efm.Model(1024, 400, seed=7)
    zero.set_params(np.zeros(zero.n_params, np.float32))
    for net, x in _tiny_cases():
        S, rev, ext = net.arrays()
        g = efm.Network(S, rev, ext)
        full = oracle.enumerate_pathways(S, rev, ext, x)
        peak = int(full.levels[:, 5].max()) if len(full.levels) else 0
        print(f"case learned tiny {net.name} x={x} peak={peak}", flush=True)
        big = efm.enumerate_learned(g, x, max(peak, 1), m)
        assert np.array_equal(big.keys, full.keys) and np.array_equal(big.flux, full.flux)
        B = max(1, peak // 3)
        canon = oracle.enumerate_pathways(S, rev, ext, x, frontier_cap=B)
        lr0 = efm.enumerate_learned(g, x, B, zero)
        assert np.array_equal(lr0.keys, canon.keys) and np.array_equal(lr0.flux, canon.flux)
        assert lr0.status == canon.status
        lr = efm.enumerate_learned(g, x, B, m)
        fk = {tuple(k): tuple(f) for k, f in zip(full.keys.tolist(), full.flux.tolist())}
        for k, f in zip(lr.keys.tolist(), lr.flux.tolist()):
            assert fk[tuple(k)] == tuple(f)


def test_learned_traversal_on_a_larger_network():
    net = netgen.learn_member(300001)
    x = net.targets[0]
    S, rev, ext = net.arrays()
    g, plain = _plain(net, x, 16)
    m = efm.Model(1024, 400, seed=8)
    print("case learned learn/300001 budget above the frontier", flush=True)
    big = efm.enumerate_learned(g, x, 1 << 24, m, depth_cap=16, unique_cap=1 << 25)
    assert np.array_equal(big.keys, plain.keys) and np.array_equal(big.flux, plain.flux)
    zero = efm.Model(1024, 400, seed=8)
    zero.set_params(np.zeros(zero.n_params, np.float32))
    flux = {tuple(k): tuple(f) for k, f in zip(plain.keys.tolist(), plain.flux.tolist())}
    for B in (1 << 10, 1 << 14):
        print(f"case learned learn/300001 budget {B}", flush=True)
        canon = efm.enumerate_pathways(g, x, depth_cap=16, frontier_cap=B, unique_cap=1 << 22)
        lr0 = efm.enumerate_learned(g, x, B, zero, depth_cap=16, unique_cap=1 << 22)
        assert np.array_equal(lr0.keys, canon.keys)
        assert [lv["kept"] for lv in lr0.levels] == [lv["kept"] for lv in canon.levels]
        r = efm.enumerate_learned(g, x, B, m, depth_cap=16, unique_cap=1 << 22)
        assert r.status & efm.FRONTIER_TRUNCATED
        assert all(lv["kept"] <= B for lv in r.levels)
        for k, f in zip(r.keys.tolist(), r.flux.tolist()):
            assert flux[tuple(k)] == tuple(f)
        if r.keys.shape[0]:
            check_result(S, rev, ext, x, r.keys, r.flux, 16)


def test_learned_rejects_bad_input():
    net = netgen.learn_member(300001)
    g = efm.Network(*net.arrays())
    small = efm.Model(32, 40, seed=0)          # 64 reactions do not fit 32 input bits
    with pytest.raises(efm.EfmError) as e:
        efm.enumerate_learned(g, net.targets[0], 100, small, depth_cap=8)
    assert e.value.code == efm.EINVAL
    m = efm.Model(1024, 400, seed=0)
    with pytest.raises(efm.EfmError) as e:
        efm.enumerate_learned(g, net.targets[0], 0, m, depth_cap=8)
    assert e.value.code == efm.EINVAL
    with pytest.raises(efm.EfmError) as e:
        efm.enumerate_learned(g, 0, 10, m, depth_cap=8)     # internal metabolite
    assert e.value.code == efm.EINVAL


def test_trained_ordering_beats_canonical_truncation():
    """The gain of the trained network: on held-out networks of the learned
    workload, at the same budget, the learned ordering recovers more of the
    exhaustive pathway set than the canonical truncation."""
    D, UC = 14, 1 << 25
    tr = efm.Traces(1024, 400, capacity=1 << 21)
    for i in range(10):
        net = netgen.learn_member(200000 + i)
        g = efm.Network(*net.arrays())
        for x in net.targets:
            try:
                tr.collect(g, x, depth_cap=D, unique_cap=UC, pos_max=500, neg_per_pos=3.0, neg_min=200,
                           seed=i * 7 + x)
            except efm.EfmError:
                pass                        # a capacity overflowed: skip this run
    n, pos = tr.info()
    print(f"case learned gain: {n} records, {pos} positive", flush=True)
    assert pos > 1000
    m = efm.Model(1024, 400, seed=0)
    st = m.train(tr, epochs=6, batch=1024, lr=2e-3, seed=0)
    assert st["loss_last"] < st["loss_first"]
    hl = hc = total = 0
    for i in range(8):
        net = netgen.learn_member(300000 + i)
        g = efm.Network(*net.arrays())
        for x in net.targets:
            try:
                p = efm.enumerate_pathways(g, x, depth_cap=D, unique_cap=UC)
            except efm.EfmError:
                continue
            if p.keys.shape[0] == 0:
                continue
            P = {tuple(k) for k in p.keys.tolist()}
            B = max(256, max(lv["kept"] for lv in p.levels) // 256)
            lr = efm.enumerate_learned(g, x, B, m, depth_cap=D, unique_cap=UC)
            cn = efm.enumerate_pathways(g, x, depth_cap=D, frontier_cap=B, unique_cap=UC)
            hl += len(P & {tuple(k) for k in lr.keys.tolist()})
            hc += len(P & {tuple(k) for k in cn.keys.tolist()})
            total += len(P)
    print(f"case learned gain: learned {hl} canonical {hc} of {total}", flush=True)
    assert total > 0
    assert hl > 2 * hc + 10
