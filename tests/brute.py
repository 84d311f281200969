"""Brute-force constructions of the 1-skeleton on tiny inputs (numpy only).

Independent of both the oracle and the GPU library; used to pin the oracle.

* ``vertices`` enumerates every candidate set of D zero entries (box faces and
  neurons) together with every activation pattern of the hidden neurons below
  the deepest zero entry, solves the resulting D x D affine system, and keeps
  the points that the true forward pass confirms: inside the box, exactly the D
  chosen entries vanish. A vertex is a 0-cell, i.e. a point with D zeros in its
  sign-vector (Sec. 3.3 / 4.1 of the paper), so this is the definition written
  out.
* ``edges_by_midpoint`` pairs vertices that share D-1 zeros with no +/-
  conflict and whose midpoint carries the join sign-vector (Sec. 3.5, 4.2.2).
* ``arrangement_edges`` (one hidden layer only) walks each line cut out by D-1
  hyperplanes/box faces and links consecutive vertices on it.
"""
from __future__ import annotations

import itertools

import numpy as np

ZERO_TOL = 1e-9
SIGN_TOL = 1e-9


def entry_count(widths, include_output=False):
    L = len(widths) - 1
    nsub = L if include_output else L - 1
    return 2 * widths[0] + sum(widths[1:1 + nsub])


def forward_all(net, x):
    """All pre-activations at the rows of x, [n, sum N_l] (plain numpy)."""
    h = np.atleast_2d(np.asarray(x, np.float64))
    outs = []
    L = len(net.W)
    for l in range(L):
        z = h @ net.W[l].T + net.b[l]
        outs.append(z)
        h = np.maximum(z, 0.0)
    return np.concatenate(outs, axis=1)


def entry_values(net, lo, hi, x, include_output=False):
    """Values whose signs make the sign-vector: box half-spaces, then neurons."""
    x = np.atleast_2d(x)
    D = x.shape[1]
    box = np.empty((x.shape[0], 2 * D))
    box[:, 0::2] = x - lo
    box[:, 1::2] = hi - x
    z = forward_all(net, x)
    M = entry_count(net.widths, include_output)
    return np.concatenate([box, z], axis=1)[:, :M]


def sign_vector(vals, tol=ZERO_TOL):
    s = np.sign(vals).astype(np.int8)
    s[np.abs(vals) < tol] = 0
    return s


def _layer_of_entries(widths, include_output):
    D = widths[0]
    L = len(widths) - 1
    nsub = L if include_output else L - 1
    lay = [0] * (2 * D)
    for l in range(1, nsub + 1):
        lay += [l] * widths[l]
    return np.array(lay)


def _affine_maps(net, pattern, upto_layer, D):
    """Affine maps (G, c) of the pre-activations of layers 1..upto_layer, given
    on/off ``pattern`` (dict layer -> bool array) for the hidden layers below."""
    G = np.eye(D)
    c = np.zeros(D)
    maps = []
    for l in range(1, upto_layer + 1):
        Gz = net.W[l - 1] @ G
        cz = net.W[l - 1] @ c + net.b[l - 1]
        maps.append((Gz, cz))
        if l < upto_layer:
            on = pattern[l].astype(np.float64)
            G = Gz * on[:, None]
            c = cz * on
    return maps


def vertices(net, lo, hi, include_output=False):
    """All vertices of the complex on the box: (X [V,D], S [V,M] int8)."""
    widths = list(net.widths)
    D = widths[0]
    M = entry_count(widths, include_output)
    lay = _layer_of_entries(widths, include_output)
    found = {}
    for Zs in itertools.combinations(range(M), D):
        deep = int(max(lay[list(Zs)]))
        # box faces of the same coordinate on both sides can't meet
        free_layers = list(range(1, deep))
        n_free = sum(widths[l] for l in free_layers)
        for bits in range(1 << n_free):
            pattern = {}
            off = 0
            for l in free_layers:
                pattern[l] = np.array([(bits >> (off + i)) & 1 for i in range(widths[l])], bool)
                off += widths[l]
            maps = _affine_maps(net, pattern, max(deep, 1), D) if deep >= 1 else []
            A = np.zeros((D, D))
            r = np.zeros(D)
            for k, e in enumerate(Zs):
                if e < 2 * D:
                    j = e // 2
                    A[k, j] = 1.0
                    r[k] = lo[j] if e % 2 == 0 else hi[j]
                else:
                    l = lay[e]
                    i = e - (2 * D + sum(widths[1:l]))
                    Gz, cz = maps[l - 1]
                    A[k] = Gz[i]
                    r[k] = -cz[i]
            if abs(np.linalg.det(A)) < 1e-12:
                continue
            x = np.linalg.solve(A, r)
            if np.any(x < lo - 1e-12) or np.any(x > hi + 1e-12):
                continue
            vals = entry_values(net, lo, hi, x, include_output)[0]
            # snap box coordinates (they are exact in the complex)
            zmask = np.abs(vals) < ZERO_TOL
            if zmask.sum() != D or not all(zmask[e] for e in Zs):
                continue
            s = sign_vector(vals)
            key = s.tobytes()
            if key not in found:
                xs = x.copy()
                for e in Zs:
                    if e < 2 * D:
                        xs[e // 2] = lo[e // 2] if e % 2 == 0 else hi[e // 2]
                found[key] = (xs, s)
        # end patterns
    X = np.array([v[0] for v in found.values()]).reshape(-1, D)
    S = np.array([v[1] for v in found.values()], dtype=np.int8).reshape(-1, M)
    return X, S


def join(sa, sb):
    """Entry-wise join of sign-vectors; returns (join, conflict_mask)."""
    j = np.where(sa == 0, sb, sa)
    conflict = (sa != 0) & (sb != 0) & (sa != sb)
    return j.astype(np.int8), conflict


def edges_by_midpoint(net, lo, hi, X, S, include_output=False):
    """Edges among the given vertices (index pairs i<j)."""
    D = X.shape[1]
    out = []
    Z = S == 0
    for i in range(len(S)):
        shared = (Z[i] & Z).sum(1)
        for j in np.nonzero(shared == D - 1)[0]:
            if j <= i:
                continue
            jn, conf = join(S[i], S[j])
            if conf.any():
                continue
            mid = 0.5 * (X[i] + X[j])
            vals = entry_values(net, lo, hi, mid, include_output)[0]
            ok = True
            for e in range(len(jn)):
                if jn[e] == 0:
                    ok &= abs(vals[e]) < 1e-7
                else:
                    ok &= np.sign(vals[e]) == jn[e] and abs(vals[e]) > 1e-12
            if ok:
                out.append((i, j))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def arrangement_edges(X, S):
    """One hidden layer: link consecutive vertices on each line of D-1 zeros."""
    D = X.shape[1]
    Z = S == 0
    M = S.shape[1]
    edges = set()
    for sub in itertools.combinations(range(M), D - 1) if D > 1 else [()]:
        on = np.all(Z[:, list(sub)], axis=1) if sub else np.ones(len(S), bool)
        idx = np.nonzero(on)[0]
        if len(idx) < 2:
            continue
        P = X[idx]
        c = P.mean(0)
        u, s, vt = np.linalg.svd(P - c)
        d = vt[0]
        order = idx[np.argsort((P - c) @ d)]
        for a, b in zip(order[:-1], order[1:]):
            edges.add((min(a, b), max(a, b)))
    return np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)


def planar_face_count(X, edges):
    """Number of faces (including the outer one) of a connected plane graph,
    by tracing half-edges around each face."""
    V = len(X)
    nbrs = [[] for _ in range(V)]
    for a, b in edges:
        nbrs[a].append(b)
        nbrs[b].append(a)
    order = []
    for v in range(V):
        ang = [np.arctan2(X[w, 1] - X[v, 1], X[w, 0] - X[v, 0]) for w in nbrs[v]]
        order.append([nbrs[v][k] for k in np.argsort(ang)])
    pos = [{w: k for k, w in enumerate(order[v])} for v in range(V)]
    seen = set()
    faces = 0
    for a, b in edges:
        for u, v in ((a, b), (b, a)):
            if (u, v) in seen:
                continue
            faces += 1
            cu, cv = u, v
            while (cu, cv) not in seen:
                seen.add((cu, cv))
                k = pos[cv][cu]
                w = order[cv][(k - 1) % len(order[cv])]
                cu, cv = cv, w
    return faces


def regions_by_perturbation(S, edges, D, m=None):
    """Sign-vectors of all regions, by perturbing every zero of every edge
    (Sec. 4.1: each zero to + and -, domain zeros (the first m entries, 2D for
    the box) only to +)."""
    m = 2 * D if m is None else m
    regs = set()
    for a, b in edges:
        jn, conf = join(S[a], S[b])
        assert not conf.any()
        zs = np.nonzero(jn == 0)[0]
        choices = [([1] if e < m else [1, -1]) for e in zs]
        for combo in itertools.product(*choices):
            r = jn.copy()
            r[zs] = combo
            regs.add(r.tobytes())
    return regs


def arrangement_counts_3d(W, b, lo, hi):
    """Vertex and edge counts of the 1-skeleton cut out of a 3-D box by the planes
    W x + b = 0 (one hidden layer), counted directly, for hundreds of planes.

    Vertices: the 8 corners; one per (plane, box edge) crossing; one per (pair of
    planes, box face) whose intersection line meets the open face; one per triple
    of planes whose common point lies in the open box. Edges from the degrees:
    a vertex with z zero box entries has degree 2D - z (Sec. 4.1 at k = 0), so
    E = (3*8 + 4*n_edge + 5*n_face + 6*n_inner) / 2."""
    W = np.asarray(W, np.float64)
    b = np.asarray(b, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    n = len(b)
    assert W.shape == (n, 3)
    n_edge = 0
    for k in range(3):                       # box edges along axis k
        o = [a for a in range(3) if a != k]
        for u in (lo[o[0]], hi[o[0]]):
            for v in (lo[o[1]], hi[o[1]]):
                p0 = np.zeros(3)
                p1 = np.zeros(3)
                p0[o[0]] = p1[o[0]] = u
                p0[o[1]] = p1[o[1]] = v
                p0[k], p1[k] = lo[k], hi[k]
                z0, z1 = W @ p0 + b, W @ p1 + b
                n_edge += int(np.sum(z0 * z1 < 0))
    ii, jj = np.triu_indices(n, 1)
    n_face = 0
    for k in range(3):                       # faces x_k = lo_k / hi_k
        o = [a for a in range(3) if a != k]
        for c in (lo[k], hi[k]):
            A = np.stack([W[ii][:, o], W[jj][:, o]], axis=1)          # [P, 2, 2]
            r = -np.stack([b[ii] + W[ii, k] * c, b[jj] + W[jj, k] * c], axis=1)
            det = A[:, 0, 0] * A[:, 1, 1] - A[:, 0, 1] * A[:, 1, 0]
            y0 = (r[:, 0] * A[:, 1, 1] - A[:, 0, 1] * r[:, 1]) / det
            y1 = (A[:, 0, 0] * r[:, 1] - r[:, 0] * A[:, 1, 0]) / det
            inside = (y0 > lo[o[0]]) & (y0 < hi[o[0]]) & (y1 > lo[o[1]]) & (y1 < hi[o[1]])
            n_face += int(np.sum(inside))
    n_inner = 0
    for i in range(n - 2):                   # triples i < j < k, one i at a time
        jk = np.array(list(itertools.combinations(range(i + 1, n), 2)), dtype=np.int64).reshape(-1, 2)
        if len(jk) == 0:
            continue
        A = np.stack([np.broadcast_to(W[i], (len(jk), 3)), W[jk[:, 0]], W[jk[:, 1]]], axis=1)
        r = -np.stack([np.full(len(jk), b[i]), b[jk[:, 0]], b[jk[:, 1]]], axis=1)
        x = np.linalg.solve(A, r[..., None])[..., 0]
        n_inner += int(np.sum(np.all((x > lo) & (x < hi), axis=1)))
    V = 8 + n_edge + n_face + n_inner
    E = (3 * 8 + 4 * n_edge + 5 * n_face + 6 * n_inner) // 2
    return V, E


# ------------------------------------------------ a domain of half-spaces

def simplex_halfspaces(corners):
    """(A, c) with A x + c the barycentric coordinates of x for the corners P_0..P_D
    (rows of ``corners``): entry i is 1 at P_i and 0 on the facet opposite it."""
    P = np.asarray(corners, np.float64)
    D = P.shape[1]
    T = np.hstack([P, np.ones((D + 1, 1))])      # [D+1, D+1]: row i = (P_i, 1)
    Ti = np.linalg.inv(T)                        # lambda(x) = (x, 1) @ Ti
    return Ti[:D].T.copy(), Ti[D].copy()


def domain_entry_values(net, A, c, x, include_output=False):
    """Domain entries A x + c, then every subdivided neuron."""
    x = np.atleast_2d(x)
    z = forward_all(net, x)
    n = entry_count(net.widths, include_output) - 2 * x.shape[1]
    return np.concatenate([x @ A.T + c, z[:, :n]], axis=1)


def vertices_halfspaces(net, A, c, include_output=False):
    """All vertices of the complex on the domain {A x + c >= 0}: every D-subset of
    entries (domain facets and neurons) under every activation pattern below the
    deepest one, solved and confirmed by the forward pass (D zeros exactly)."""
    widths = list(net.widths)
    D = widths[0]
    m = len(c)
    L = len(widths) - 1
    nsub = L if include_output else L - 1
    lay = np.array([0] * m + sum(([l] * widths[l] for l in range(1, nsub + 1)), []))
    M = len(lay)
    found = {}
    for Zs in itertools.combinations(range(M), D):
        deep = int(max(lay[list(Zs)]))
        free_layers = list(range(1, deep))
        n_free = sum(widths[l] for l in free_layers)
        for bits in range(1 << n_free):
            pattern = {}
            off = 0
            for l in free_layers:
                pattern[l] = np.array([(bits >> (off + i)) & 1 for i in range(widths[l])], bool)
                off += widths[l]
            maps = _affine_maps(net, pattern, max(deep, 1), D) if deep >= 1 else []
            Am = np.zeros((D, D))
            r = np.zeros(D)
            for k, e in enumerate(Zs):
                if e < m:
                    Am[k] = A[e]
                    r[k] = -c[e]
                else:
                    l = lay[e]
                    i = e - (m + sum(widths[1:l]))
                    Gz, cz = maps[l - 1]
                    Am[k] = Gz[i]
                    r[k] = -cz[i]
            if abs(np.linalg.det(Am)) < 1e-12:
                continue
            x = np.linalg.solve(Am, r)
            vals = domain_entry_values(net, A, c, x, include_output)[0]
            if np.any(vals[:m] < -1e-9):
                continue
            zmask = np.abs(vals) < ZERO_TOL
            if zmask.sum() != D or not all(zmask[e] for e in Zs):
                continue
            s = sign_vector(vals)
            found.setdefault(s.tobytes(), (x, s))
    X = np.array([v[0] for v in found.values()]).reshape(-1, D)
    S = np.array([v[1] for v in found.values()], dtype=np.int8).reshape(-1, M)
    return X, S


def edges_by_midpoint_halfspaces(net, A, c, X, S, include_output=False):
    """Edges among the given vertices of a half-space domain (index pairs i<j):
    D-1 shared zeros, no +/- conflict, midpoint carrying the join."""
    D = X.shape[1]
    out = []
    Z = S == 0
    for i in range(len(S)):
        shared = (Z[i] & Z).sum(1)
        for j in np.nonzero(shared == D - 1)[0]:
            if j <= i:
                continue
            jn, conf = join(S[i], S[j])
            if conf.any():
                continue
            vals = domain_entry_values(net, A, c, 0.5 * (X[i] + X[j]), include_output)[0]
            on = jn == 0
            if np.all(np.abs(vals[on]) < 1e-7) and np.all((np.sign(vals[~on]) == jn[~on]) & (np.abs(vals[~on]) > 1e-12)):
                out.append((i, j))
    return np.array(out, dtype=np.int64).reshape(-1, 2)
