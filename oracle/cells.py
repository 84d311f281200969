"""Higher cells of the complex by repeated perturbation -- TEST INFRASTRUCTURE ONLY.

Sec. 4.1 of the paper: a k-cell's parents are obtained by perturbing each zero
of its sign-vector to + and to - (zeros of the domain's half-spaces only to +,
toward the inside), and every (k+1)-cell is a parent of some k-cell. Starting
from the edges (the sign-vector of an edge is the join of its two vertices',
Sec. 3.5), this gives the 2-faces, then the 3-cells, ..., up to the regions
(D-cells, no zeros left). Plain Python sets of sign-vectors: for small cases.
"""
from __future__ import annotations

import numpy as np


def edge_signs(S, edges):
    """Sign-vector of each edge: the join of its endpoints' (equal signs stay,
    0 joins s to s; the endpoints of an edge never conflict)."""
    a, b = S[edges[:, 0]], S[edges[:, 1]]
    return np.where(a == 0, b, a).astype(np.int8)


def parents(rows, m, mutation=0):
    """The set of (k+1)-cells above the given k-cells (rows: iterable of int8 arrays).
    mutation (test-only planted mistakes): 1 = domain zeros also to -, 2 = every
    zero only to +."""
    out = set()
    for r in rows:
        for e in np.nonzero(r == 0)[0]:
            if mutation == 1:
                signs = (1, -1)
            elif mutation == 2:
                signs = (1,)
            else:
                signs = (1,) if e < m else (1, -1)
            for sg in signs:
                p = r.copy()
                p[e] = sg
                out.add(p.tobytes())
    return out


def face_counts(S, edges, D, m, mutation=0):
    """(f_0, f_1, ..., f_D) and the regions' sign-vectors [f_D, M] (sorted rows)."""
    S = np.asarray(S, np.int8)
    edges = np.asarray(edges, np.int64)
    counts = [len(S), len(edges)]
    level = [r for r in edge_signs(S, edges)] if len(edges) else []
    if D == 1:
        return counts, np.array(level, np.int8).reshape(-1, S.shape[1])
    for k in range(1, D):
        nxt = parents(level, m, mutation)
        counts.append(len(nxt))
        level = [np.frombuffer(x, np.int8) for x in sorted(nxt)]
    return counts, np.array(level, np.int8).reshape(-1, S.shape[1])
