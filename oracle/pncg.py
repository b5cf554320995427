"""2x2 subspace step, restart ratio, safe step and the PNCG loop (FP64).

Test infrastructure (see the package docstring).

* Subspace step (Section 4.2; supplement Section 2): p(mu, nu) = -mu z + nu p_k
  minimises Q = g^T p + 1/2 p^T H~ p.  The oracle forms the three entries
  z^T H~ z, z^T H~ p_k, p_k^T H~ p_k with explicit products by the assembled
  H~ and solves the 2x2 system of supplement Eq. (10) by Gaussian elimination
  with partial pivoting.  Near-singular systems (supplement Section 2.4.3:
  |Delta| < eps_sing max(A11 A22, eps_abs)) fall back to mu = 1, nu = 0.
* Restart iteration (Algorithm 1): mu = g^T z / z^T H~ z, nu = 0.  The
  supplement's alternative (mu = 1 on the very first iteration) is not used;
  mu = 1, nu = 0 is also taken when z^T H~ z <= 0.
* Restart ratio (Section 4.3): r_k = |g_{k+1}^T z_k| / (g_{k+1}^T z_{k+1}).
* Safe step (Section 4.4, supplement Section 3): the cubic CCD of the paper
  reduces to a linear time of contact for affine stencils.  Candidate c
  closes at the rate s_c = -sum_j grad_{c,j} . p_j (the relative
  displacement of its vertices, so a common translation does not count) and
  gets a_c = max(0, min(1, 0.9 d_c / s_c)) when s_c > 0; a subdomain takes
  the minimum over the candidates touching it (Algorithm 1, per-subdomain
  steps).  A common step keeps every d_c >= 0.1 d_c; where the subdomains of
  one stencil move with different steps and the combined motion would bring
  it below 0.05 d_c, the steps of those subdomains are halved, repeatedly
  (at most 16 rounds), so that only the critical subdomains are damped.
"""
from __future__ import annotations

import numpy as np


def solve2(A, b):
    """2x2 Gaussian elimination with partial pivoting."""
    A = np.array(A, np.float64)
    b = np.array(b, np.float64)
    if abs(A[1, 0]) > abs(A[0, 0]):
        A = A[::-1].copy()
        b = b[::-1].copy()
    l = A[1, 0] / A[0, 0]
    a22 = A[1, 1] - l * A[0, 1]
    b2 = b[1] - l * b[0]
    y = b2 / a22
    x = (b[0] - A[0, 1] * y) / A[0, 0]
    return np.array([x, y])


def subspace_step(g, z, p, Hmul, restart, eps_sing=1e-12, eps_abs=1e-300):
    """Returns (mu, nu, p_next, fallback, A11, A12, A22)."""
    Hz = Hmul(z)
    A11 = float(z @ Hz)
    gz = float(g @ z)
    if restart:
        if A11 > 0:
            mu, nu, fb = gz / A11, 0.0, False
        else:
            mu, nu, fb = 1.0, 0.0, True
        return mu, nu, -mu * z, fb, A11, 0.0, 0.0
    Hp = Hmul(p)
    A12 = float(z @ Hp)
    A22 = float(p @ Hp)
    gp = float(g @ p)
    det = A11 * A22 - A12 * A12
    if abs(det) < eps_sing * max(A11 * A22, eps_abs):
        return 1.0, 0.0, -z, True, A11, A12, A22
    mu, nu = solve2([[A11, -A12], [-A12, A22]], [gz, -gp])
    return float(mu), float(nu), -mu * z + nu * p, False, A11, A12, A22


# Comparison direction rules (Section 5, search-direction study): classic
# nonlinear CG with a preconditioner, p = alpha d, d = -z + beta d_prev.
BETA_FR, BETA_CD, BETA_DK = 1, 2, 3


def beta_coefficient(rule, g, g_prev, z, z_prev, d_prev):
    """beta of the comparison rules, preconditioned (z = P g), or None when
    its denominator is not positive.  The paper names the rules without
    formulas; these are the published ones with g^T g replaced by g^T z:

    * Fletcher-Reeves (1964): g^T z / (g_prev^T z_prev);
    * conjugate descent (Fletcher 1987): g^T z / (-d_prev^T g_prev);
    * Dai-Kou (2013), the member tau = s^T y / s^T s of their family:
      y^T z / (d^T y) - (y^T P y / d^T y) (d^T g) / (d^T y), y = g - g_prev,
      with P y = z - z_prev.
    """
    g, g_prev, z, z_prev, d_prev = (np.asarray(a, np.float64) for a in (g, g_prev, z, z_prev, d_prev))
    if rule == BETA_FR:
        num, den = float(g @ z), float(g_prev @ z_prev)
        return num / den if den > 0 else None
    if rule == BETA_CD:
        num, den = float(g @ z), -float(d_prev @ g_prev)
        return num / den if den > 0 else None
    if rule == BETA_DK:
        y = g - g_prev
        dy = float(d_prev @ y)
        if not dy > 0:
            return None
        return float(y @ z) / dy - (float(y @ (z - z_prev)) / dy) * (float(d_prev @ g) / dy)
    raise ValueError("unknown rule %r" % (rule,))


def beta_step(rule, g, g_prev, z, z_prev, d_prev, Hmul, restart):
    """One direction of a comparison rule: d = -z + beta d_prev (beta = 0 on
    a restart), alpha minimising g^T (alpha d) + 1/2 alpha^2 d^T H~ d, and
    the step p = alpha d that the safe step then scales per subdomain.
    Safeguards (the reading used where the rules need them): a denominator
    that is not positive, or a d that is not a descent direction
    (g^T d >= 0), gives d = -z; d^T H~ d <= 0 gives alpha = 1.  Either sets
    the fallback flag.  Returns (alpha, beta, d, p, fallback)."""
    fb = False
    beta = 0.0
    if not restart:
        b = beta_coefficient(rule, g, g_prev, z, z_prev, d_prev)
        if b is None:
            fb = True
        else:
            beta = b
    d = -z + beta * d_prev if beta != 0.0 else -np.asarray(z, np.float64)
    gd = float(g @ d)
    if not restart and not gd < 0:
        beta, fb = 0.0, True
        d = -np.asarray(z, np.float64)
        gd = float(g @ d)
    dHd = float(d @ Hmul(d))
    if dHd > 0:
        alpha = -gd / dHd
    else:
        alpha, fb = 1.0, True
    return alpha, beta, d, alpha * d, fb


def restart_ratio(g_new, z_prev, z_new):
    return abs(float(g_new @ z_prev)) / float(g_new @ z_new)


SAFE_ROUNDS = 16


def safe_alpha(hier, idx, grad, d, p):
    """Per-subdomain step sizes (D,) for affine candidate stencils
    (Section 4.4; supplement Section 3).  Along p a stencil's distance
    changes at the rate sum_j grad_j . p_j (its vertices moving together:
    the relative displacement, independent of the frame); if it closes, its
    step is 0.9 of the time to contact, capped at 1 (and 0 for a stencil
    already at d <= 0).  Each subdomain takes the smallest step of the
    stencils touching it; subdomains whose different steps would together
    close a stencil are then damped (halved) until none does.  If
    SAFE_ROUNDS rounds leave such a stencil, every subdomain takes instead
    the bound that holds for any mix of per-vertex steps: a stencil whose
    vertices close at the rates s_j = max(0, -grad_j . p_j) takes
    min(1, 0.9 d / sum_j s_j), each subdomain the smallest over its
    stencils, so that no stencil comes below 0.1 d whatever steps its
    vertices take up to that bound."""
    P = np.asarray(p).reshape(-1, 3)
    D = hier.num_subdomains(0)
    alpha = np.ones(D)
    for c in range(idx.shape[0]):
        rate = 0.0
        for j in range(4):
            v = idx[c, j]
            if v >= 0:
                rate -= float(grad[c, 3 * j:3 * j + 3] @ P[v])
        if rate <= 0.0:
            continue
        a = max(0.0, min(1.0, 0.9 * d[c] / rate))
        for j in range(4):
            v = idx[c, j]
            if v >= 0:
                sd = hier.subdomain_of_vertex(v)
                alpha[sd] = min(alpha[sd], a)
    # Vertices of one stencil in different subdomains move with different
    # steps: while the combined motion would bring a stencil below 0.05 of
    # its distance, halve the steps of every subdomain such a stencil touches.
    sub = np.where(idx >= 0, hier.rank[np.maximum(idx, 0)] // 32, -1)

    def violating(a):
        marked = np.zeros(D, bool)
        for c in range(idx.shape[0]):
            if not d[c] > 0.0:
                continue
            dn = d[c]
            for j in range(4):
                v = idx[c, j]
                if v >= 0:
                    dn += a[sub[c, j]] * float(grad[c, 3 * j:3 * j + 3] @ P[v])
            if dn < 0.05 * d[c]:
                marked[sub[c][sub[c] >= 0]] = True
        return marked

    for _ in range(SAFE_ROUNDS):
        marked = violating(alpha)
        if not marked.any():
            return alpha
        alpha[marked] *= 0.5
    if not violating(alpha).any():
        return alpha
    # the rounds did not separate every stencil: the bound for any mix
    safe = np.ones(D)
    for c in range(idx.shape[0]):
        closing = 0.0
        for j in range(4):
            v = idx[c, j]
            if v >= 0:
                closing += max(0.0, -float(grad[c, 3 * j:3 * j + 3] @ P[v]))
        if closing <= 0.0:
            continue
        a = max(0.0, min(1.0, 0.9 * d[c] / closing))
        for j in range(4):
            if idx[c, j] >= 0:
                safe[sub[c, j]] = min(safe[sub[c, j]], a)
    return safe


def step_positions(hier, x, p, alpha):
    """x + S_d^T alpha_d S_d p for every subdomain (Algorithm 1)."""
    a = alpha[hier.rank // 32]
    return (np.asarray(x).reshape(-1, 3) + a[:, None] * np.asarray(p).reshape(-1, 3)).reshape(-1)


def ccd_safe_alpha(hier, x, p, radius, pairs, kinds, dist):
    """Per-subdomain steps on point-triangle / edge-edge pairs (Algorithm 1's
    ConservativeCCD and per-subdomain alpha_d; Section 4.4; supplement
    Section 3).  Each subdomain starts at the smallest CCD step along p
    (``oracle.ccd.pair_step``) of the candidate pairs with a vertex in it,
    capped at radius / (2 max_v |p_v|) (candidates are every pair closer
    than radius; no two vertices approach each other by more than the cap
    allows, so the others cannot meet).  A pair whose vertices lie in
    subdomains with different steps is checked by the CCD along its
    vertices' actual displacements; while one finds a root before 1, the
    steps of its subdomains are halved (at most SAFE_ROUNDS rounds).  If a
    pair is left after that, every subdomain takes the smallest step (one
    common step along p, which the CCD covers)."""
    from . import ccd
    X = np.asarray(x, np.float64).reshape(-1, 3)
    P = np.asarray(p, np.float64).reshape(-1, 3)
    D = hier.num_subdomains(0)
    alpha = np.ones(D)
    sub = hier.rank[np.asarray(pairs, np.int64)] // 32 if len(pairs) else np.zeros((0, 4), np.int64)
    for i in range(len(pairs)):
        a = ccd.pair_step(X[pairs[i]], P[pairs[i]], kinds[i], dist[i])
        for s in sub[i]:
            alpha[s] = min(alpha[s], a)
    pmax = float(np.max(np.linalg.norm(P, axis=1))) if P.size else 0.0
    if pmax > 0.0:
        alpha = np.minimum(alpha, min(1.0, radius / (2.0 * pmax)))
    common = alpha.min()   # one step along p for every subdomain

    def violating(a):
        marked = np.zeros(D, bool)
        for i in range(len(pairs)):
            s = a[sub[i]]
            if np.all(s == s[0]):
                continue
            step = ccd.pair_step(X[pairs[i]], s[:, None] * P[pairs[i]], kinds[i], dist[i])
            if step < 1.0:
                marked[sub[i]] = True
        return marked

    for _ in range(SAFE_ROUNDS):
        marked = violating(alpha)
        if not marked.any():
            return alpha
        alpha = np.where(marked, 0.5 * alpha, alpha)
    if not violating(alpha).any():
        return alpha
    return np.full(D, common)
