"""Contact distances of point-triangle and edge-edge pairs (FP64).

Test infrastructure (see the package docstring).

The barrier of Section 3.1 acts on the distance d_c of a contact pair;
the projected contact Hessian of Section 4.1 and the update columns
u = sqrt(k) n of supplement Eq. (11) use n = grad d_c.  The paper gives no formula for d_c; it is read here as the
unsigned Euclidean distance between the two primitives (a point and a
triangle, or two segments), and its gradient as the envelope-theorem one:
with closest points c_1 = sum_j w_j y_j on the first primitive and
c_2 = sum_j w_j y_j on the second, n_hat = (c_1 - c_2) / d and
d/dy_j d = w_j n_hat on the first primitive, -w_j n_hat on the second
(point-triangle: the point is the first primitive, weights 1; the
triangle's are the barycentric weights of the closest point).

Method here: every sub-simplex that can hold the minimiser is tried (the
interior stationary point when it is feasible, each edge by clamped
projection, each vertex) and the smallest distance is kept.  This is the
definition of the minimum over the product of the two simplices, evaluated
candidate by candidate.

Types (closest features):
* point-triangle: 0, 1, 2 = vertex T0, T1, T2; 3, 4, 5 = edge T0T1, T1T2,
  T2T0; 6 = face.
* edge-edge: 3 a + b, with a (first edge) and b (second edge) each 0 = the
  edge's first vertex, 1 = its second vertex, 2 = interior.
"""
from __future__ import annotations

import numpy as np

PT, EE = 0, 1


def _seg_closest(p, a, b):
    """Weight s in [0, 1] of the closest point a + s (b - a) to p."""
    e = b - a
    ee = float(e @ e)
    if ee == 0.0:
        return 0.0
    return min(1.0, max(0.0, float((p - a) @ e) / ee))


def point_triangle(p, t0, t1, t2):
    """(d, weights (w0, w1, w2) of the closest point, type)."""
    p, t0, t1, t2 = (np.asarray(v, np.float64) for v in (p, t0, t1, t2))
    cands = []
    # interior: minimise |p - t0 - u e1 - v e2|^2 (normal equations)
    e1, e2, r = t1 - t0, t2 - t0, p - t0
    G = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
    if abs(np.linalg.det(G)) > 1e-300 and np.linalg.cond(G) < 1e14:
        u, v = np.linalg.solve(G, np.array([e1 @ r, e2 @ r]))
        if u > 0.0 and v > 0.0 and u + v < 1.0:
            cands.append(((1.0 - u - v, u, v), 6))
    # edges (open segments) and vertices
    T = (t0, t1, t2)
    for k, (i, j) in enumerate(((0, 1), (1, 2), (2, 0))):
        s = _seg_closest(p, T[i], T[j])
        if 0.0 < s < 1.0:
            w = [0.0, 0.0, 0.0]
            w[i], w[j] = 1.0 - s, s
            cands.append((tuple(w), 3 + k))
    for i in range(3):
        w = [0.0, 0.0, 0.0]
        w[i] = 1.0
        cands.append((tuple(w), i))
    best = None
    for w, ty in cands:
        c = w[0] * t0 + w[1] * t1 + w[2] * t2
        d = float(np.linalg.norm(p - c))
        if best is None or d < best[0]:
            best = (d, w, ty)
    return best


def edge_edge(a0, a1, b0, b1):
    """(d, (s, t), type): closest points a0 + s (a1 - a0), b0 + t (b1 - b0)."""
    a0, a1, b0, b1 = (np.asarray(v, np.float64) for v in (a0, a1, b0, b1))
    u, v, r = a1 - a0, b1 - b0, a0 - b0
    cands = []
    G = np.array([[u @ u, -(u @ v)], [-(u @ v), v @ v]])
    if abs(np.linalg.det(G)) > 1e-300 and np.linalg.cond(G) < 1e14:
        s, t = np.linalg.solve(G, np.array([-(u @ r), v @ r]))
        if 0.0 < s < 1.0 and 0.0 < t < 1.0:
            cands.append((s, t))
    # the four sides of the (s, t) square
    for s in (0.0, 1.0):
        cands.append((s, _seg_closest(a0 + s * u, b0, b1)))
    for t in (0.0, 1.0):
        cands.append((_seg_closest(b0 + t * v, a0, a1), t))
    best = None
    for s, t in cands:
        d = float(np.linalg.norm(a0 + s * u - b0 - t * v))
        if best is None or d < best[0]:
            best = (d, (s, t))
    d, (s, t) = best

    def feat(q):
        return 0 if q == 0.0 else (1 if q == 1.0 else 2)

    return d, (s, t), 3 * feat(s) + feat(t)


def pair_distance(x4, kind):
    """(d, grad (12,), type) of one pair, x4: (4, 3) in pair order."""
    X = np.asarray(x4, np.float64)
    if kind == PT:
        d, w, ty = point_triangle(*X)
        wt = np.array([1.0, -w[0], -w[1], -w[2]])
        c1, c2 = X[0], w[0] * X[1] + w[1] * X[2] + w[2] * X[3]
    else:
        d, (s, t), ty = edge_edge(*X)
        wt = np.array([1.0 - s, s, -(1.0 - t), -t])
        c1, c2 = (1.0 - s) * X[0] + s * X[1], (1.0 - t) * X[2] + t * X[3]
    g = np.zeros(12)
    if d > 0.0:
        n = (c1 - c2) / d
        g = np.concatenate([wt[j] * n for j in range(4)])
    return d, g, ty


def contact_distances(x, pairs, kinds):
    """Distances (m,), gradients (m, 12) and types (m,) of all pairs."""
    X = np.asarray(x, np.float64).reshape(-1, 3)
    m = pairs.shape[0]
    d = np.zeros(m)
    g = np.zeros((m, 12))
    ty = np.zeros(m, np.int64)
    for i in range(m):
        d[i], g[i], ty[i] = pair_distance(X[pairs[i]], kinds[i])
    return d, g, ty
