"""Brute-force elementary-pathway enumeration straight from Definitions 1-3.

Independent of the oracle (different language, different algorithm): every
reaction subset E is tried.  E supports an elementary mode iff the internal-row
submatrix S_int[:, E] has a one-dimensional null space whose vector has no zero
entry and feasible signs.  (Definition 2 for v; Definition 3 for minimality: with
a null space of dimension one no balanced mode lives on a smaller support, and a
dimension of two or more always yields one on a smaller support.)

Exactness.  Ranks and the null vector's zero pattern are computed modulo the
prime p = 2^31 - 1 for all subsets at once (batched Gauss-Jordan in numpy).  The
test asserts that p exceeds Hadamard's bound on every square minor of S_int, so a
minor vanishes mod p exactly when it vanishes over the rationals: the mod-p rank
equals the rational rank, and a null-vector entry (a maximal minor, by Cramer's
rule) is zero mod p exactly when it is zero; scaled by the pivot minor, the mod-p
null vector is the vector of maximal minors, whose symmetric residues are the
exact integers.  `nullspace_fraction` (exact rationals) cross-checks that lift in
the tests.

Subsets in which an internal metabolite is touched by exactly one reaction of E
are skipped first: that reaction's flux would be forced to zero.  This is a
necessary condition only, so nothing is lost.
"""
from __future__ import annotations

import math
from fractions import Fraction
from math import gcd

import numpy as np

P = 2**31 - 1


def hadamard_bound(Sint: np.ndarray) -> float:
    """Upper bound on |det| of any square submatrix: product of the largest
    column norms (log-space)."""
    norms = np.sqrt((Sint.astype(np.float64) ** 2).sum(axis=0))
    norms = np.sort(norms[norms > 0])[::-1]
    k = min(Sint.shape)
    return float(np.exp(np.log(np.maximum(norms[:k], 1.0)).sum()))


def _powmod(a: np.ndarray, e: int) -> np.ndarray:
    r = np.ones_like(a)
    b = a % P
    while e:
        if e & 1:
            r = (r * b) % P
        b = (b * b) % P
        e >>= 1
    return r


def _batched_rref(A: np.ndarray, colmask: np.ndarray):
    """Gauss-Jordan mod P of every matrix A[b] (rows x cols), restricted to the
    columns with colmask[b, c] set.  Returns (A reduced, rank, pivot column of each
    rank row (-1 unused), product of the pivots before normalisation).  Only
    multiples of pivot rows are added to other rows, so that product is, up to
    sign, the minor on the pivot rows and pivot columns."""
    B, R, C = A.shape
    rank = np.zeros(B, np.int64)
    det = np.ones(B, np.int64)
    pivcol = np.full((B, R), -1, np.int64)
    rows = np.arange(R)
    bidx = np.arange(B)
    for c in range(C):
        cand = (A[:, :, c] != 0) & (rows[None, :] >= rank[:, None]) & colmask[:, c][:, None]
        has = cand.any(axis=1)
        if not has.any():
            continue
        b = bidx[has]
        pr = np.argmax(cand[has], axis=1)
        rk = rank[has]
        tmp = A[b, pr, :].copy()
        A[b, pr, :] = A[b, rk, :]
        A[b, rk, :] = tmp
        det[b] = (det[b] * A[b, rk, c]) % P
        inv = _powmod(A[b, rk, c], P - 2)
        A[b, rk, :] = (A[b, rk, :] * inv[:, None]) % P
        prow = A[b, rk, :]                                   # (nb, C)
        f = A[b, :, c].copy()                                # (nb, R)
        f[np.arange(b.size), rk] = 0
        A[b] = (A[b] - (f[:, :, None] * prow[:, None, :]) % P) % P
        pivcol[b, rk] = c
        rank[b] += 1
    return A, rank, pivcol, det


def nullspace_fraction(M, ncols):
    """Basis of {v : M v = 0} over the rationals (Gauss-Jordan)."""
    A = [[Fraction(x) for x in row] for row in M]
    pivots = []
    r = 0
    for c in range(ncols):
        p = next((i for i in range(r, len(A)) if A[i][c] != 0), None)
        if p is None:
            continue
        A[r], A[p] = A[p], A[r]
        inv = 1 / A[r][c]
        A[r] = [x * inv for x in A[r]]
        for i in range(len(A)):
            if i != r and A[i][c] != 0:
                fct = A[i][c]
                A[i] = [a - fct * b for a, b in zip(A[i], A[r])]
        pivots.append(c)
        r += 1
    basis = []
    for fc in (c for c in range(ncols) if c not in pivots):
        v = [Fraction(0)] * ncols
        v[fc] = Fraction(1)
        for row, pc in enumerate(pivots):
            v[pc] = -A[row][fc]
        basis.append(v)
    return basis


def primitive(v):
    den = 1
    for x in v:
        den = den * x.denominator // gcd(den, x.denominator)
    iv = [int(x * den) for x in v]
    g = 0
    for x in iv:
        g = gcd(g, abs(x))
    return [x // g for x in iv]


def circuits(S, ext, depth_cap: int = 0, chunk: int = 40000):
    """Supports whose internal-row submatrix has a one-dimensional null space with
    no zero entry: [(support as python int, column list, primitive integer null vector on those
    columns)], any target."""
    S = np.asarray(S, dtype=np.int64)
    m, n = S.shape
    if n > 22:
        raise ValueError("brute force is for tiny networks")
    internal = [i for i in range(m) if not ext[i]]
    Sint = S[internal]
    assert hadamard_bound(Sint) < P, "prime too small for exact mod-p ranks"
    D = depth_cap if depth_cap > 0 else n
    subsets = np.arange(1, 1 << n, dtype=np.int64)
    ok = np.ones(subsets.shape, bool)
    for i in range(len(internal)):
        mask = sum(1 << j for j in range(n) if Sint[i, j] != 0)
        x = subsets & mask
        ok &= ~((x != 0) & ((x & (x - 1)) == 0))
    bits = ((subsets[:, None] >> np.arange(n)[None, :]) & 1).astype(bool)
    ok &= bits.sum(axis=1) <= D
    subsets, bits = subsets[ok], bits[ok]
    found = []
    R = Sint.shape[0]
    for s0 in range(0, subsets.size, chunk):
        sb, cm = subsets[s0:s0 + chunk], bits[s0:s0 + chunk]
        A = np.broadcast_to(Sint % P, (sb.size,) + Sint.shape).copy()
        A[~np.broadcast_to(cm[:, None, :], A.shape)] = 0
        A, rank, pivcol, det = _batched_rref(A, cm)
        one = np.nonzero(rank == cm.sum(axis=1) - 1)[0]
        if one.size == 0:
            continue
        pm = np.zeros((one.size, n), bool)
        pc = pivcol[one]
        rr, cc = np.nonzero(pc >= 0)
        pm[rr, pc[rr, cc]] = True
        free = cm[one] & ~pm
        assert (free.sum(axis=1) == 1).all()
        fcol = np.argmax(free, axis=1)
        vals = A[one, :, :][np.arange(one.size), :, fcol]         # (nb, R): -v on pivot rows
        full = ((vals % P != 0) | (np.arange(R)[None, :] >= rank[one][:, None])).all(axis=1)
        # Cramer: det * v is the vector of signed maximal minors, each below the
        # Hadamard bound < P/2, so its symmetric residues are the exact integers.
        for q in np.nonzero(full)[0].tolist():
            b = int(one[q])
            cols = np.nonzero(cm[b])[0].tolist()
            w = np.zeros(n, np.int64)
            w[fcol[q]] = det[b]
            for row in range(int(rank[b])):
                w[pivcol[b, row]] = (-vals[q, row] * det[b]) % P
            w = np.where(w > P // 2, w - P, w)
            g = 0
            for x in w.tolist():
                g = gcd(g, abs(int(x)))
            vec = [int(w[j]) // g for j in cols]
            found.append((int(sb[b]), cols, vec))
    return found


def elementary_pathways(S, rev, ext, target: int, depth_cap: int = 0, circ=None):
    """All (support as a python int, dense flux list) that produce `target`,
    sorted by the support read as an integer.  `circ` may pass precomputed
    circuits(S, ext, depth_cap)."""
    S = np.asarray(S, dtype=np.int64)
    m, n = S.shape
    internal = [i for i in range(m) if not ext[i]]
    Sint = S[internal]
    if circ is None:
        circ = circuits(S, ext, depth_cap)
    out = []
    for E, cols, v in circ:
        if not any(S[target, j] != 0 for j in cols):
            continue
        signs = {1 if v[k] > 0 else -1 for k, j in enumerate(cols) if not rev[j]}
        if len(signs) > 1:
            continue
        if signs == {-1}:
            v = [-x for x in v]
        prod = sum(int(S[target, j]) * v[k] for k, j in enumerate(cols))
        if not signs and prod < 0:                # all reversible: orient to produce target
            v = [-x for x in v]
            prod = -prod
        if prod <= 0:
            continue
        dense = [0] * n
        for k, j in enumerate(cols):
            dense[j] = v[k]
        out.append((E, dense))
    out.sort(key=lambda t: t[0])
    return out
