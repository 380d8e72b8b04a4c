"""CPU oracle of the learned frontier ordering (test infrastructure).

Plain numpy in float64, written from the definitions; it shares no code with the
GPU library.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg import it.

What it covers:

* the canonical relabelling of a network's reactions and internal metabolites
  around a target (positions by breadth-first distance from the target's
  producing reactions, then by decreasing degree, then by index), which makes
  the model's inputs comparable across networks;
* the sparse input of a partial pathway P: one unit entry per reaction of P at
  its relabelled position, and one entry per internal metabolite i with a
  non-zero imbalance count u_i = clamp(#{r in P: S_ir > 0} - #{r in P: S_ir < 0},
  -7, 7): each metabolite owns two input rows, in_bits + 2 * (relabelled i) for a
  surplus and the next one for a deficit, and the entry is |u_i| / 8 on the row of
  its sign (so that one linear unit can sum the magnitudes);
* the trace label of a partial pathway: 1 iff some elementary flux mode found by
  the plain traversal contains it (a sub-pathway that closes into a balanced one);
* the three-layer perceptron  s = w3 . relu(W2^T relu(W1^T x + b1) + b2) + b3,
  its mean weighted binary cross-entropy on logits, the gradients of that loss,
  and one Adam step with bias correction.

The paper prints no numbers for any of this (the learned ordering is a systems
addition on top of its traversal, which orders the frontier it describes in its
Algorithm 3 and its Theorem 1 budget discussion), so the learned scores are
parity-unpinned against the paper; the functions are pinned against library
routines (torch autograd in float64, torch's Adam, scikit-learn's log loss),
finite differences and hand-worked examples.
"""
from __future__ import annotations

from collections import deque

import numpy as np

UNREACHED = 1 << 30


# ------------------------------------------------------------------ relabelling

def relabel(S, rev, ext, x):
    """Positions of reactions (rpos[r]) and internal metabolites (mpos[k], k-th
    internal row) around target metabolite x.

    Distances are breadth-first over the bipartite graph of internal metabolites
    and reactions: the reactions with S[x, r] != 0 are at distance 0, an internal
    metabolite touched by a reaction at distance d is at d + 1, a reaction
    touching a metabolite at distance d is at d + 1.  Reaction degree = number of
    internal metabolites it touches; metabolite degree = number of reactions
    touching it.  Position = rank under (distance, -degree, index)."""
    S = np.asarray(S)
    m, n = S.shape
    internal = [i for i in range(m) if not ext[i]]
    mi = len(internal)
    Si = S[internal, :] if mi else np.zeros((0, n), S.dtype)
    rdist = [UNREACHED] * n
    mdist = [UNREACHED] * mi
    q = deque()
    for r in range(n):
        if S[x, r] != 0:
            rdist[r] = 0
            q.append(("r", r))
    while q:
        kind, v = q.popleft()
        if kind == "r":
            for k in range(mi):
                if Si[k, v] != 0 and mdist[k] == UNREACHED:
                    mdist[k] = rdist[v] + 1
                    q.append(("m", k))
        else:
            for r in range(n):
                if Si[v, r] != 0 and rdist[r] == UNREACHED:
                    rdist[r] = mdist[v] + 1
                    q.append(("r", r))
    rdeg = [int(np.count_nonzero(Si[:, r])) for r in range(n)]
    mdeg = [int(np.count_nonzero(Si[k, :])) for k in range(mi)]
    rorder = sorted(range(n), key=lambda r: (rdist[r], -rdeg[r], r))
    morder = sorted(range(mi), key=lambda k: (mdist[k], -mdeg[k], k))
    rpos = np.empty(n, np.int64)
    mpos = np.empty(mi, np.int64)
    for p, r in enumerate(rorder):
        rpos[r] = p
    for p, k in enumerate(morder):
        mpos[k] = p
    return rpos, mpos


# ------------------------------------------------------------------- features

def features(S, ext, reactions, rpos, mpos, in_bits):
    """Sparse input of the partial pathway with reaction set `reactions`:
    a list of (row, code) pairs, reactions first in increasing reaction index,
    then internal metabolites in increasing internal index.  code 0 = a reaction
    bit (value 1); code c in 1..7 = an imbalance of magnitude c (value c / 8) on
    the metabolite's surplus row (u > 0) or deficit row (u < 0)."""
    S = np.asarray(S)
    internal = [i for i in range(S.shape[0]) if not ext[i]]
    rs = sorted(set(int(r) for r in reactions))
    out = [(int(rpos[r]), 0) for r in rs]
    for k, row in enumerate(internal):
        c = 0
        for r in rs:
            if S[row, r] > 0:
                c += 1
            elif S[row, r] < 0:
                c -= 1
        u = max(-7, min(7, c))
        if u != 0:
            out.append((in_bits + 2 * int(mpos[k]) + (1 if u < 0 else 0), abs(u)))
    return out


def encode(entries):
    """16-bit entry words (row << 4 | code), the record format of the traces."""
    return np.array([(row << 4) | code for row, code in entries], np.uint16)


def decode(words):
    w = np.asarray(words, np.int64)
    return [(int(v >> 4), int(v & 15)) for v in w]


def code_value(code):
    return 1.0 if code == 0 else code / 8.0


def dense(records, F):
    """Dense float64 input matrix of a list of entry lists."""
    X = np.zeros((len(records), F))
    for i, ent in enumerate(records):
        for row, code in ent:
            X[i, row] += code_value(code)
    return X


def keys_to_reactions(key_words):
    """Reaction indices of a bitset given as uint64 words (reaction r = bit r & 63
    of word r >> 6)."""
    out = []
    for w, word in enumerate(np.asarray(key_words, np.uint64).tolist()):
        b = 0
        while word:
            if word & 1:
                out.append(64 * w + b)
            word >>= 1
            b += 1
    return out


# --------------------------------------------------------------------- labels

def label(state_keys, found_keys):
    """1 where the state (row of uint64 words) is a subset of some found pathway."""
    st = np.asarray(state_keys, np.uint64)
    fd = np.asarray(found_keys, np.uint64)
    out = np.zeros(len(st), np.uint8)
    for i, s in enumerate(st):
        for f in fd:
            if np.all((s & ~f[:s.shape[0]]) == 0):
                out[i] = 1
                break
    return out


# ------------------------------------------------------------------ perceptron

PARAM_ORDER = ("W1", "b1", "W2", "b2", "w3", "b3")


def shapes(F, H):
    return {"W1": (F, H), "b1": (H,), "W2": (H, H), "b2": (H,), "w3": (H,), "b3": (1,)}


def unflatten(flat, F, H):
    flat = np.asarray(flat, np.float64)
    P, off = {}, 0
    for k in PARAM_ORDER:
        shp = shapes(F, H)[k]
        size = int(np.prod(shp))
        P[k] = flat[off:off + size].reshape(shp)
        off += size
    if off != flat.size:
        raise ValueError("parameter vector has the wrong length")
    return P


def flatten(P):
    return np.concatenate([np.asarray(P[k], np.float64).ravel() for k in PARAM_ORDER])


def forward(P, X):
    z1 = X @ P["W1"] + P["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ P["W2"] + P["b2"]
    a2 = np.maximum(z2, 0.0)
    s = a2 @ P["w3"] + P["b3"][0]
    return {"z1": z1, "a1": a1, "z2": z2, "a2": a2, "s": s}


def _softplus(t):
    return np.logaddexp(0.0, t)


def _sigmoid(t):
    return 0.5 * (1.0 + np.tanh(0.5 * t))


def loss_and_grad(P, X, y, pos_weight=1.0):
    """Mean over the batch of  pw * y * softplus(-s) + (1 - y) * softplus(s),
    and its gradient with respect to every parameter (backpropagation through the
    two rectifiers; the derivative of a rectifier at exactly 0 is taken as 0)."""
    y = np.asarray(y, np.float64)
    B = X.shape[0]
    f = forward(P, X)
    s = f["s"]
    loss = float(np.mean(pos_weight * y * _softplus(-s) + (1.0 - y) * _softplus(s)))
    sig = _sigmoid(s)
    g = (pos_weight * y * (sig - 1.0) + (1.0 - y) * sig) / B          # dL/ds
    G = {"b3": np.array([g.sum()]), "w3": f["a2"].T @ g}
    dz2 = np.outer(g, P["w3"]) * (f["z2"] > 0)
    G["W2"] = f["a1"].T @ dz2
    G["b2"] = dz2.sum(0)
    dz1 = (dz2 @ P["W2"].T) * (f["z1"] > 0)
    G["W1"] = X.T @ dz1
    G["b1"] = dz1.sum(0)
    return loss, G, f


def adam_step(P, G, M, V, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1) with bias-corrected moments."""
    nP, nM, nV = {}, {}, {}
    for k in P:
        nM[k] = beta1 * M[k] + (1.0 - beta1) * G[k]
        nV[k] = beta2 * V[k] + (1.0 - beta2) * G[k] * G[k]
        mh = nM[k] / (1.0 - beta1 ** t)
        vh = nV[k] / (1.0 - beta2 ** t)
        nP[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return nP, nM, nV
