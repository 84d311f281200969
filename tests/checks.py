"""Invariant checks and canonical forms for 1-skeletons (test helpers).

A complex is given as coordinates X [V, D] (float64), sign-vectors S [V, M]
(int8 in {+1, 0, -1}) and edges [E, 2]. Nothing here imports the oracle or the
GPU library.
"""
from __future__ import annotations

import numpy as np

from brute import entry_values, join


def unpack_signs(packed: np.ndarray, widths, include_output=False, m=None) -> np.ndarray:
    """Packed rows ([V, Wd] uint64) to int8 sign-vectors [V, M] in {+1, 0, -1}.

    Packing of include/pcx.h: 2 bits per entry, 00 = 0, 01 = +, 10 = -; domain
    entry e (m of them: 2D for the box, D + 1 for a simplex) in word 0 at bits
    2e; neuron i of the l-th subdivided layer in word lw_l + i // 32 at bits
    2 (i % 32), with lw_1 = 1, lw_{l+1} = lw_l + ceil(N_l / 32)."""
    packed = np.ascontiguousarray(packed, dtype=np.uint64)
    D = int(widths[0])
    m = 2 * D if m is None else m
    L = len(widths) - 1
    nsub = L if include_output else L - 1
    cols = [(0, 2 * e) for e in range(m)]
    lw = 1
    for l in range(1, nsub + 1):
        n = int(widths[l])
        cols += [(lw + i // 32, 2 * (i % 32)) for i in range(n)]
        lw += -(-n // 32)
    assert packed.shape[1] == lw, f"expected {lw} words per row, got {packed.shape[1]}"
    word = np.array([c[0] for c in cols])
    shift = np.array([c[1] for c in cols], dtype=np.uint64)
    codes = (packed[:, word] >> shift) & np.uint64(3)
    if np.any(codes == 3):
        raise AssertionError("invalid sign code 11")
    out = np.zeros(codes.shape, np.int8)
    out[codes == 1] = 1
    out[codes == 2] = -1
    # bits outside every entry must be clear
    used = np.zeros(lw, dtype=np.uint64)
    for w, sh in cols:
        used[w] |= np.uint64(3) << np.uint64(sh)
    assert not np.any(packed & ~used), "bits set outside the entries"
    return out


def canonical(X, S, edges):
    """Vertices sorted by sign-vector bytes; edges as sorted (min, max) pairs
    of canonical ids. Returns (X, S, edges, perm) with perm[old] = new."""
    S = np.ascontiguousarray(S, dtype=np.int8)
    keys = S.view(np.dtype((np.void, S.shape[1]))).ravel()
    order = np.argsort(keys, kind="stable")
    perm = np.empty(len(order), np.int64)
    perm[order] = np.arange(len(order))
    E = perm[np.asarray(edges, np.int64)]
    E = np.sort(E, axis=1)
    E = E[np.lexsort((E[:, 1], E[:, 0]))] if len(E) else E.reshape(0, 2)
    return X[order], S[order], E, perm


def assert_same_complex(A, B, coord_tol=1e-10):
    """Bit-exact sign-vectors, counts and canonical incidence; coordinates to tol."""
    XA, SA, EA, _ = canonical(*A)
    XB, SB, EB, _ = canonical(*B)
    assert SA.shape == SB.shape, f"vertex/entry counts differ: {SA.shape} vs {SB.shape}"
    assert np.array_equal(SA, SB), "sign-vectors differ"
    assert EA.shape == EB.shape, f"edge counts differ: {EA.shape} vs {EB.shape}"
    assert np.array_equal(EA, EB), "edge incidence differs"
    err = np.max(np.abs(XA - XB)) if len(XA) else 0.0
    assert err <= coord_tol, f"coordinates differ by {err}"


def check_invariants(net, lo, hi, X, S, edges, include_output=False, zero_tol=1e-9, full=True, sample=None):
    """Properties that hold for the 1-skeleton of any generic instance. sample:
    run the forward-pass checks on that many random vertices and edges only
    (the combinatorial checks always cover everything)."""
    V, M = S.shape
    D = X.shape[1]
    edges = np.asarray(edges, np.int64)
    # a vertex is a 0-cell: exactly D zeros (Sec. 4.1)
    zc = (S == 0).sum(1)
    assert np.all(zc == D), f"vertices with != D zeros: {np.nonzero(zc != D)[0][:5]}"
    # interior cells are + on the domain entries; no vertex outside the box
    assert np.all(S[:, :2 * D] >= 0), "negative box entry"
    for j in range(D):
        at_lo = S[:, 2 * j] == 0
        at_hi = S[:, 2 * j + 1] == 0
        assert np.all(X[at_lo, j] == lo[j]) and np.all(X[at_hi, j] == hi[j]), "box coordinate not exact"
        inner = ~(at_lo | at_hi)
        assert np.all((X[inner, j] > lo[j]) & (X[inner, j] < hi[j])), "vertex outside the box"
    # distinct cells have distinct sign-vectors
    keys = np.ascontiguousarray(S).view(np.dtype((np.void, M))).ravel()
    assert len(np.unique(keys)) == V, "duplicate sign-vectors"
    # edges: D-1 shared zeros, no +/- conflict (Sec. 4.1, 4.2.2)
    a, b = edges[:, 0], edges[:, 1]
    assert np.all(a != b)
    shared = ((S[a] == 0) & (S[b] == 0)).sum(1)
    assert np.all(shared == D - 1), "edge without D-1 shared zeros"
    conflict = (S[a] != 0) & (S[b] != 0) & (S[a] != S[b])
    assert not conflict.any(), "edge endpoints in conflict"
    ek = np.sort(edges, axis=1)
    assert len(np.unique(ek, axis=0)) == len(ek), "duplicate edges"
    # vertex degree = 2D - (number of zero box entries), Sec. 4.1 at k = 0
    zbox = (S[:, :2 * D] == 0).sum(1)
    deg = np.bincount(edges.ravel(), minlength=V)
    assert np.array_equal(deg, 2 * D - zbox), "degree != 2D - z_box"
    assert 2 * len(edges) == np.sum(2 * D - zbox)
    if not full:
        return
    X_full, S_full = X, S
    if sample is not None:
        rng = np.random.default_rng(0)
        vi = rng.choice(V, size=min(sample, V), replace=False)
        X, S = X[vi], S[vi]
        ei = rng.choice(len(a), size=min(sample, len(a)), replace=False)
        Sa, Sb, Xa, Xb = S_full[a[ei]], S_full[b[ei]], X_full[a[ei]], X_full[b[ei]]
    else:
        Sa, Sb, Xa, Xb = S_full[a], S_full[b], X_full[a], X_full[b]
    # validation of Sec. 5.1.1: zero entries evaluate to ~0, signs agree elsewhere
    vals = entry_values(net, lo, hi, X, include_output)
    assert np.all(np.abs(vals[S == 0]) < zero_tol), f"max |z| at zeros {np.abs(vals[S == 0]).max()}"
    nz = S != 0
    assert np.all(np.sign(vals[nz]) == S[nz]), "forward-pass sign differs from sign-vector"
    # midpoint of each edge lies in the edge's cell: sign = join
    jn = np.where(Sa == 0, Sb, Sa)
    mid = 0.5 * (Xa + Xb)
    mv = entry_values(net, lo, hi, mid, include_output)
    assert np.all(np.abs(mv[jn == 0]) < 1e-7), "edge leaves a hyperplane it should lie on"
    assert np.all(np.sign(mv[jn != 0]) == jn[jn != 0]), "edge midpoint outside its cell"


def digest(S, edges):
    """sha256 over the canonical sign-vectors and canonical edge list."""
    import hashlib
    X = np.zeros((len(S), 1))
    _, Sc, Ec, _ = canonical(X, S, edges)
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(Sc, np.int8).tobytes())
    h.update(np.ascontiguousarray(Ec, np.int64).tobytes())
    return h.hexdigest()


def level_set(X, S, edges):
    """The output's zero level set inside a complex extracted with the output
    subdivided: vertices with 0 at the last entry, edges between two of them
    (renumbered in vertex order)."""
    keep = np.asarray(S)[:, -1] == 0
    idx = np.nonzero(keep)[0]
    new = -np.ones(len(keep), np.int64)
    new[idx] = np.arange(len(idx))
    edges = np.asarray(edges, np.int64)
    both = keep[edges[:, 0]] & keep[edges[:, 1]] if len(edges) else np.zeros(0, bool)
    return X[idx], S[idx], new[edges[both]].reshape(-1, 2)
