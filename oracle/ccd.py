"""Conservative CCD for point-triangle and edge-edge pairs (FP64).

Test infrastructure (see the package docstring).

* Lower bound (supplement Section 3): along the search direction p the
  relative displacement of any two points of the pair is at most l per unit
  step.  The standard bound (Eq. (23)) adds the largest displacement on each
  side; the frame-invariant bound takes the largest relative displacement
  of a vertex pair across the primitives (Eq. (29) point-triangle,
  Eq. (31) edge-edge), which is never larger.  alpha_l = d_min / l with
  d_min = 0.9 dist (see ``pair_step``).
* Coplanarity cubic (supplement Section 3.4): f(t) is the signed volume of
  the tetrahedron spanned by the four vertices at x + t p.  Its coefficients
  are obtained here by evaluating the determinant at t = 0, 1, 2, 3 and
  solving the 4x4 Vandermonde system (the cubic is exact, so four samples
  fix it).
* SafeBisect (supplement Algorithm 1) with the update of y_s taken in the
  branch that advances x_s; CubicSafe (supplement Algorithm 2): the
  interval [max(0, alpha_l), 1] is cut at the critical points of f into
  monotonic pieces and the first piece whose ends differ in sign is bisected
  sixteen times toward the safe side.
"""
from __future__ import annotations

import numpy as np

PT, EE = 0, 1


def l_tight(pairs_p, kind):
    """Eq. (29) / (31): largest relative displacement between a vertex of
    one primitive and a vertex of the other.  pairs_p: (4,3)."""
    p = np.asarray(pairs_p, np.float64)
    if kind == PT:
        return max(np.linalg.norm(p[0] - p[j]) for j in (1, 2, 3))
    return max(np.linalg.norm(p[i] - p[j]) for i in (0, 1) for j in (2, 3))


def l_original(pairs_p, kind):
    """Eq. (23) and its edge-edge analogue: the largest displacement on each
    side, added."""
    n = np.linalg.norm(np.asarray(pairs_p, np.float64), axis=1)
    if kind == PT:
        return n[0] + n[1:].max()
    return n[:2].max() + n[2:].max()


def volume(x4):
    """Signed volume (times 6) of the tetrahedron of the four points."""
    x4 = np.asarray(x4, np.float64)
    return float(np.linalg.det(np.stack([x4[1] - x4[0], x4[2] - x4[0], x4[3] - x4[0]])))


def cubic_coefficients(x4, p4):
    """[d, c, b, a] of f(t) = a t^3 + b t^2 + c t + d = volume(x + t p)."""
    ts = np.array([0.0, 1.0, 2.0, 3.0])
    f = np.array([volume(np.asarray(x4) + t * np.asarray(p4)) for t in ts])
    V = np.vander(ts, 4, increasing=True)
    return np.linalg.solve(V, f)


def _f(coef, t):
    d, c, b, a = coef
    return ((a * t + b) * t + c) * t + d


def _sign(v):
    return int(v > 0) - int(v < 0)


def safe_bisect(coef, xs, xu, ys, yu):
    """Sixteen halvings of [xs, xu] keeping f(xs) on the side of ys."""
    for _ in range(16):
        xm = 0.5 * (xs + xu)
        ym = _f(coef, xm)
        if _sign(ys) != _sign(ym):
            xu = xm
        else:
            xs = xm
            ys = ym
    return xs


def cubic_safe(coef, alpha_l):
    """Largest safe step in [alpha_l, 1] for the cubic (supplement
    Algorithm 2)."""
    d, c, b, a = (float(v) for v in coef)
    coef = (d, c, b, a)
    if alpha_l >= 1.0:
        return 1.0
    x = max(0.0, alpha_l)
    y = _f(coef, x)
    if y == 0.0:
        return x
    y1 = _f(coef, 1.0)
    disc = b * b - 3.0 * a * c
    if disc > 0.0:
        q = -(b + np.copysign(np.sqrt(disc), b))
        r1 = q / (3.0 * a) if a != 0.0 else np.inf
        r2 = c / q if q != 0.0 else np.inf
        xa, xb = min(r1, r2), max(r1, r2)
        if x < xa < 1.0:
            ya = _f(coef, xa)
            if _sign(y) != _sign(ya):
                return safe_bisect(coef, x, xa, y, ya)
            x, y = xa, ya
        if x < xb < 1.0:
            yb = _f(coef, xb)
            if _sign(y) != _sign(yb):
                if x > alpha_l:
                    return x
                return safe_bisect(coef, x, xb, y, yb)
            x, y = xb, yb
    elif disc == 0.0 and a != 0.0:
        xi = -b / (3.0 * a)
        if x < xi < 1.0:
            yi = _f(coef, xi)
            if _sign(y) != _sign(yi):
                return safe_bisect(coef, x, xi, y, yi)
            x, y = xi, yi
    if _sign(y) != _sign(y1):
        if x > alpha_l:
            return x
        return safe_bisect(coef, x, 1.0, y, y1)
    return 1.0


D_MIN_FRACTION = 0.9


def pair_step(x4, p4, kind, dist):
    """Safe step of one pair: alpha_l = d_min / l_tight, then CubicSafe.
    The supplement leaves d_min open; the reading here is d_min = 0.9 dist
    (the conservative fraction of additive CCD), so that a coplanarity root
    before alpha_l is always a crossing of the plane away from the other
    primitive (the pair is still at least 0.1 dist apart there) and a pair
    that meets exactly at dist / l_tight (a pure approach along the
    contact normal) is found by CubicSafe instead of being skipped."""
    l = l_tight(p4, kind)
    alpha_l = D_MIN_FRACTION * dist / l if l > 0.0 else np.inf
    return cubic_safe(cubic_coefficients(x4, p4), alpha_l)


def ccd_steps(hier, x, p, pairs, kinds, dist):
    """Per-pair steps and per-subdomain minima (Algorithm 1's alpha_d)."""
    X = np.asarray(x, np.float64).reshape(-1, 3)
    P = np.asarray(p, np.float64).reshape(-1, 3)
    m = pairs.shape[0]
    a = np.array([pair_step(X[pairs[i]], P[pairs[i]], kinds[i], dist[i]) for i in range(m)])
    alpha = np.ones(hier.num_subdomains(0))
    for i in range(m):
        for v in pairs[i]:
            sd = hier.subdomain_of_vertex(v)
            alpha[sd] = min(alpha[sd], a[i])
    return a, alpha
