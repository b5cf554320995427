"""ComputeConstraintSet of Algorithm 1 by brute force (FP64).

Test infrastructure (see the package docstring).

The active contact set is every point-triangle pair (a surface vertex and
a surface triangle not containing it) and every edge-edge pair (two
surface edges without a common vertex, each pair once) whose distance
(``oracle.contact``) is below dhat.  All pairs are considered; a pair is
skipped without computing its distance only when the distance between the
axis-aligned boxes of its two primitives is already >= dhat, which is a
lower bound of the primitives' distance because each box contains its
primitive.
"""
from __future__ import annotations

import numpy as np

from . import contact

CHUNK = 4096


def box_distance(lo1, hi1, lo2, hi2):
    """Euclidean distance between axis-aligned boxes (broadcasting)."""
    gap = np.maximum(0.0, np.maximum(lo1 - hi2, lo2 - hi1))
    return np.sqrt(np.sum(gap * gap, axis=-1))


def _candidates(lo_a, hi_a, lo_b, hi_b, dhat):
    out = []
    for s in range(0, lo_a.shape[0], CHUNK):
        bd = box_distance(lo_a[s:s + CHUNK, None], hi_a[s:s + CHUNK, None], lo_b[None], hi_b[None])
        i, j = np.nonzero(bd < dhat)
        out.append(np.stack([i + s, j], 1))
    return np.concatenate(out) if out else np.zeros((0, 2), np.int64)


def constraint_set(x, verts, tris, edges, dhat):
    """Returns (pairs (m, 4), kinds (m,), d (m,)) sorted by (kind, ids)."""
    X = np.asarray(x, np.float64).reshape(-1, 3)
    verts = np.asarray(verts, np.int64)
    tris = np.asarray(tris, np.int64)
    edges = np.asarray(edges, np.int64)
    P = X[verts]
    T = X[tris]
    E = X[edges]
    rows = []
    # point-triangle
    for a, b in _candidates(P, P, T.min(1), T.max(1), dhat):
        v, t = verts[a], tris[b]
        if v in t:
            continue
        ids = np.array([v, t[0], t[1], t[2]])
        d = contact.pair_distance(X[ids], contact.PT)[0]
        if d < dhat:
            rows.append((contact.PT, ids, d))
    # edge-edge, each unordered pair once (first edge index smaller)
    for a, b in _candidates(E.min(1), E.max(1), E.min(1), E.max(1), dhat):
        if a >= b:
            continue
        e1, e2 = edges[a], edges[b]
        if len({e1[0], e1[1], e2[0], e2[1]}) < 4:
            continue
        ids = np.array([e1[0], e1[1], e2[0], e2[1]])
        d = contact.pair_distance(X[ids], contact.EE)[0]
        if d < dhat:
            rows.append((contact.EE, ids, d))
    if not rows:
        return np.zeros((0, 4), np.int64), np.zeros(0, np.uint8), np.zeros(0)
    kinds = np.array([r[0] for r in rows], np.uint8)
    pairs = np.stack([r[1] for r in rows])
    d = np.array([r[2] for r in rows])
    order = np.lexsort((pairs[:, 3], pairs[:, 2], pairs[:, 1], pairs[:, 0], kinds))
    return pairs[order], kinds[order], d[order]
