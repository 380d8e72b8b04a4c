"""Pins of the learned-ordering oracle (oracle/learned.py) against hand-worked
examples, library routines (torch autograd and Adam in float64, scikit-learn's
log loss) and finite differences.  CPU only."""
import numpy as np
import pytest
import torch

from oracle import learned as L


def _net5():
    """Internal A, B, C (rows 0-2), external x_in, x_out (rows 3-4).
    r0: A -> B;  r1: 2A -> B + C;  r2: A <=> x_in;  r3: B <=> x_out;  r4: C -> A."""
    S = np.zeros((5, 5), np.int64)
    S[0, 0], S[1, 0] = -1, 1
    S[0, 1], S[1, 1], S[2, 1] = -2, 1, 1
    S[0, 2], S[3, 2] = -1, 1
    S[1, 3], S[4, 3] = -1, 1
    S[2, 4], S[0, 4] = -1, 1
    rev = np.array([0, 0, 1, 1, 0], np.uint8)
    ext = np.array([0, 0, 0, 1, 1], np.uint8)
    return S, rev, ext


def test_relabel_hand_worked():
    # distances from x_out's exchange r3: r3 0; B 1; r0, r1 2; A, C 3; r2, r4 4.
    # reaction degrees r0 2, r1 3, r2 1, r3 1, r4 2 -> order r3, r1, r0, r4, r2.
    # metabolite degrees A 4, B 3, C 2 -> order B, A, C.
    S, rev, ext = _net5()
    rpos, mpos = L.relabel(S, rev, ext, 4)
    assert rpos.tolist() == [2, 1, 4, 0, 3]
    assert mpos.tolist() == [1, 0, 2]
    # from x_in's exchange r2: r2 0; A 1; r0, r1, r4 2 (degrees 2, 3, 2); B, C 3; r3 4.
    rpos, mpos = L.relabel(S, rev, ext, 3)
    assert rpos.tolist() == [2, 1, 0, 4, 3]
    assert mpos.tolist() == [0, 1, 2]


def test_relabel_unreached_last():
    S, rev, ext = _net5()
    S2 = np.zeros((6, 6), np.int64)
    S2[:5, :5] = S
    S2[5, 5] = 1          # a reaction touching only a new external row: unreachable
    ext2 = np.array([0, 0, 0, 1, 1, 1], np.uint8)
    rpos, _ = L.relabel(S2, np.zeros(6, np.uint8), ext2, 4)
    assert rpos[5] == 5


def test_features_hand_worked():
    S, rev, ext = _net5()
    rpos, mpos = L.relabel(S, rev, ext, 4)
    # P = {r0, r3}: bits r0 -> 2, r3 -> 0; A consumed once -> u = -1: magnitude 1 on
    # A's deficit row 8 + 2 * 1 + 1
    assert L.features(S, ext, [3, 0], rpos, mpos, 8) == [(2, 0), (0, 0), (11, 1)]
    # P = {r1, r3, r4}: every count cancels (signs are counted, not coefficients)
    assert L.features(S, ext, [1, 3, 4], rpos, mpos, 8) == [(1, 0), (0, 0), (3, 0)]
    # P = {r0, r1, r2, r3}: A -3 (deficit row 11), B +1 (surplus row 8), C +1 (surplus row 12)
    assert L.features(S, ext, [0, 1, 2, 3], rpos, mpos, 8) == [
        (2, 0), (1, 0), (4, 0), (0, 0), (11, 3), (8, 1), (12, 1)]


def test_features_clamp():
    # metabolite M consumed by nine reactions: count -9 clamps to -7 (deficit row, 7)
    S = np.zeros((11, 10), np.int64)
    for r in range(9):
        S[0, r] = -1
        S[1 + r, r] = 1
    S[0, 9], S[10, 9] = 1, -1
    ext = np.zeros(11, np.uint8)
    ext[10] = 1
    rpos, mpos = L.relabel(S, np.zeros(10, np.uint8), ext, 10)
    ent = L.features(S, ext, range(9), rpos, mpos, 16)
    counts = [e for e in ent if e[0] >= 16]
    assert (16 + 2 * mpos[0] + 1, 7) in counts
    assert sum(1 for e in counts if e[1] == 1 and (e[0] - 16) % 2 == 0) == 9   # the nine products
    assert L.decode(L.encode(ent)) == ent


def test_label_hand_worked():
    f = np.array([[0b1011], [0b0110]], np.uint64)
    st = np.array([[0b0011], [0b0101], [0b0110], [0b1000], [0b1111]], np.uint64)
    assert L.label(st, f).tolist() == [1, 0, 1, 1, 0]


def _hand_params():
    return {"W1": np.array([[1.0, -1.0], [0.5, 2.0], [-1.0, 1.0]]), "b1": np.array([0.0, -0.5]),
            "W2": np.array([[1.0, 0.0], [-2.0, 1.0]]), "b2": np.array([0.25, 0.0]),
            "w3": np.array([2.0, -1.0]), "b3": np.array([0.1])}


def test_forward_hand_worked():
    f = L.forward(_hand_params(), np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 1.0]]))
    # x0: z1 (1.5, 0.5), z2 (0.75, 0.5), s 1.1;  x1: z1 (-1, 0.5), z2 (-0.75, 0.5), s -0.4
    assert np.allclose(f["z1"], [[1.5, 0.5], [-1.0, 0.5]], atol=0, rtol=0)
    assert np.allclose(f["z2"], [[0.75, 0.5], [-0.75, 0.5]], atol=0, rtol=0)
    assert np.allclose(f["s"], [1.1, -0.4], atol=1e-15)


def _random_problem(seed, B=9, F=7, H=5):
    rng = np.random.default_rng(seed)
    P = {k: rng.normal(size=shp) * 0.7 for k, shp in L.shapes(F, H).items()}
    X = (rng.random((B, F)) < 0.4).astype(np.float64)
    X[:, F - 2:] = rng.integers(-7, 8, size=(B, 2)) / 8.0
    y = (rng.random(B) < 0.4).astype(np.float64)
    return P, X, y


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("pw", [1.0, 7.5])
def test_loss_and_grad_match_torch_autograd(seed, pw):
    P, X, y = _random_problem(seed)
    loss, G, _ = L.loss_and_grad(P, X, y, pw)
    T = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}
    Xt = torch.tensor(X)
    a1 = torch.relu(Xt @ T["W1"] + T["b1"])
    a2 = torch.relu(a1 @ T["W2"] + T["b2"])
    s = a2 @ T["w3"] + T["b3"][0]
    lt = torch.nn.functional.binary_cross_entropy_with_logits(
        s, torch.tensor(y), pos_weight=torch.tensor(pw, dtype=torch.float64))
    lt.backward()
    assert abs(loss - lt.item()) < 1e-12
    for k in L.PARAM_ORDER:
        assert np.allclose(G[k], T[k].grad.numpy(), rtol=1e-10, atol=1e-13), k


def test_loss_matches_sklearn_log_loss():
    from sklearn.metrics import log_loss
    P, X, y = _random_problem(11, B=40)
    loss, _, f = L.loss_and_grad(P, X, y, 1.0)
    p = 1.0 / (1.0 + np.exp(-f["s"]))
    assert abs(loss - log_loss(y, p, labels=[0, 1])) < 1e-9


@pytest.mark.parametrize("seed", range(3))
def test_grad_matches_finite_differences(seed):
    P, X, y = _random_problem(100 + seed)
    _, G, f = L.loss_and_grad(P, X, y, 3.0)
    # skip instances whose rectifiers sit within the step of a kink
    h = 1e-6
    if min(np.abs(f["z1"]).min(), np.abs(f["z2"]).min()) < 1e-3:
        pytest.skip("pre-activation too close to a kink for central differences")
    for k in L.PARAM_ORDER:
        flat = P[k].ravel()
        for j in range(flat.size):
            Pp = {q: v.copy() for q, v in P.items()}
            Pm = {q: v.copy() for q, v in P.items()}
            Pp[k].ravel()[j] += h
            Pm[k].ravel()[j] -= h
            num = (L.loss_and_grad(Pp, X, y, 3.0)[0] - L.loss_and_grad(Pm, X, y, 3.0)[0]) / (2 * h)
            assert abs(num - G[k].ravel()[j]) < 1e-7, (k, j)


def test_adam_matches_torch_optim():
    P, X, y = _random_problem(7)
    T = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}
    opt = torch.optim.Adam([T[k] for k in L.PARAM_ORDER], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    M = {k: np.zeros_like(v) for k, v in P.items()}
    V = {k: np.zeros_like(v) for k, v in P.items()}
    Q = {k: v.copy() for k, v in P.items()}
    for t in range(1, 6):
        _, G, _ = L.loss_and_grad(Q, X, y, 2.0)
        Q, M, V = L.adam_step(Q, G, M, V, t, 3e-3)
        opt.zero_grad()
        for k in L.PARAM_ORDER:
            T[k].grad = torch.tensor(L.loss_and_grad({q: T[q].detach().numpy() for q in T}, X, y, 2.0)[1][k])
        opt.step()
        for k in L.PARAM_ORDER:
            assert np.allclose(Q[k], T[k].detach().numpy(), rtol=1e-12, atol=1e-14), (t, k)


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g the bias-corrected moments are g and g^2 at every
    # step, so each update is -lr * g / (|g| + eps)
    P = {"w": np.array([0.3, -1.0, 2.0])}
    g = np.array([0.5, -2e-3, 0.0])
    M, V = {"w": np.zeros(3)}, {"w": np.zeros(3)}
    Q = P
    for t in range(1, 8):
        Q, M, V = L.adam_step(Q, {"w": g}, M, V, t, 0.01)
    expect = P["w"] - 7 * 0.01 * g / (np.abs(g) + 1e-8)
    assert np.allclose(Q["w"], expect, rtol=1e-12, atol=1e-15)


def test_flatten_roundtrip():
    P, _, _ = _random_problem(3)
    flat = L.flatten(P)
    assert flat.size == 7 * 5 + 5 + 25 + 5 + 5 + 1
    Q = L.unflatten(flat, 7, 5)
    for k in L.PARAM_ORDER:
        assert np.array_equal(P[k], Q[k])
