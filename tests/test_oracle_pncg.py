"""Pins of the oracle's subspace step, restart ratio and safe step.

Anchors: numpy.linalg.solve for the 2x2 system, stationarity of the
quadratic model checked by finite differences in (mu, nu), the descent
property g^T p < 0, the degenerate direction p = c z, the textbook
equivalence with preconditioned CG on an SPD quadratic, and the safety
property of the affine step bound.
"""
import numpy as np
import pytest

from oracle import ccd, mas, pncg
from oracle import contact as C
from paper_2604_19892_amd import synth


def spd(rng, n, cond=1e3):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q @ np.diag(np.geomspace(1, cond, n)) @ Q.T


def test_two_by_two_matches_lapack_and_is_stationary():
    rng = np.random.default_rng(0)
    n = 30
    A = spd(rng, n)
    g, z, p = rng.standard_normal((3, n))
    mu, nu, pn, fb, A11, A12, A22 = pncg.subspace_step(g, z, p, lambda v: A @ v, restart=False)
    assert not fb
    ref = np.linalg.solve([[z @ A @ z, -(z @ A @ p)], [-(p @ A @ z), p @ A @ p]], [g @ z, -(g @ p)])
    np.testing.assert_allclose([mu, nu], ref, rtol=1e-12)

    def Q(m_, n_):
        q = -m_ * z + n_ * p
        return g @ q + 0.5 * q @ A @ q

    h = 1e-5 * max(1.0, abs(mu), abs(nu))
    dQm = (Q(mu + h, nu) - Q(mu - h, nu)) / (2 * h)
    dQn = (Q(mu, nu + h) - Q(mu, nu - h)) / (2 * h)
    scale = abs(g @ z) + abs(g @ p)
    assert abs(dQm) < 1e-7 * scale and abs(dQn) < 1e-7 * scale
    # the optimum is a descent direction: g^T p = -[mu nu] A_sub [mu nu]^T < 0
    Asub = np.array([[A11, -A12], [-A12, A22]])
    sol = np.array([mu, nu])
    assert g @ pn == pytest.approx(-sol @ Asub @ sol, rel=1e-10)
    assert g @ pn < 0


def test_pivoting_path_matches_lapack():
    A = np.array([[1e-14, 2.0], [3.0, 1.0]])
    b = np.array([1.0, 2.0])
    np.testing.assert_allclose(pncg.solve2(A, b), np.linalg.solve(A, b), rtol=1e-14)


def test_fallback_on_parallel_directions():
    rng = np.random.default_rng(1)
    A = spd(rng, 10)
    g, z = rng.standard_normal((2, 10))
    mu, nu, pn, fb, *_ = pncg.subspace_step(g, z, -2.5 * z, lambda v: A @ v, restart=False)
    assert fb and mu == 1.0 and nu == 0.0
    np.testing.assert_array_equal(pn, -z)


def test_restart_iteration_is_exact_line_search():
    rng = np.random.default_rng(2)
    A = spd(rng, 12)
    g, z = rng.standard_normal((2, 12))
    mu, nu, pn, fb, *_ = pncg.subspace_step(g, z, np.zeros(12), lambda v: A @ v, restart=True)
    assert nu == 0 and not fb
    # minimiser of g^T(-mu z) + 1/2 mu^2 z^T A z
    assert mu == pytest.approx((g @ z) / (z @ A @ z), rel=1e-14)


def test_subspace_pncg_equals_pcg_on_spd_quadratic():
    """With H~ = A exact, a fixed SPD preconditioner and unit steps, the
    2D-subspace iteration reproduces preconditioned CG and terminates in at
    most n steps."""
    rng = np.random.default_rng(3)
    n = 12
    A = spd(rng, n, cond=10.0)
    Pm = np.linalg.inv(np.diag(np.diag(A)) + 0.1 * spd(rng, n, cond=10))
    Pm = 0.5 * (Pm + Pm.T)
    b = rng.standard_normal(n)
    # textbook PCG
    x = np.zeros(n)
    r = b - A @ x
    zc = Pm @ r
    d = zc.copy()
    xs_pcg = []
    for _ in range(n):
        a = (r @ zc) / (d @ A @ d)
        x = x + a * d
        r_new = r - a * (A @ d)
        z_new = Pm @ r_new
        beta = (r_new @ z_new) / (r @ zc)
        d = z_new + beta * d
        r, zc = r_new, z_new
        xs_pcg.append(x.copy())
    # 2D subspace with alpha = 1
    x = np.zeros(n)
    p = np.zeros(n)
    xs = []
    for k in range(n):
        g = A @ x - b
        z = Pm @ g
        mu, nu, p, fb, *_ = pncg.subspace_step(g, z, p, lambda v: A @ v, restart=(k == 0))
        x = x + p
        xs.append(x.copy())
    xe = np.linalg.solve(A, b)
    for k in range(n):
        assert np.linalg.norm(xs[k] - xs_pcg[k]) < 1e-10 * np.linalg.norm(xe)
    # finite termination (exact arithmetic: n steps), up to rounding
    assert np.linalg.norm(xs[-1] - xe) < 1e-10 * np.linalg.norm(xe)
    assert np.linalg.norm(xs[n // 2] - xe) > 1e-6 * np.linalg.norm(xe)


def test_restart_ratio_definition_cases():
    g = np.array([1.0, 2.0])
    assert pncg.restart_ratio(g, np.array([1.0, 0.0]), np.array([0.0, 1.0])) == pytest.approx(0.5)
    assert pncg.restart_ratio(g, np.array([-3.0, 0.0]), np.array([1.0, 1.0])) == pytest.approx(1.0)


def test_safe_step_keeps_every_stencil_apart():
    sc = synth.two_boxes_scene(n_contacts=3000, nxy=12, nz=6, active_frac=0.7)
    hier = mas.Hierarchy(sc.X, 2)
    pool = sc.pool
    rng = np.random.default_rng(4)
    x = sc.x.reshape(-1)
    p = 0.05 * rng.standard_normal(x.size)

    def dist(xx):
        xs = np.where(pool['idx'][..., None] >= 0, xx.reshape(-1, 3)[np.maximum(pool['idx'], 0)], 0)
        return (pool['grad'] * xs.reshape(-1, 12)).sum(1) - pool['off']

    d0 = dist(x)
    alpha = pncg.safe_alpha(hier, pool['idx'], pool['grad'], d0, p)
    assert np.all((alpha > 0) & (alpha <= 1))
    assert np.any(alpha < 1)
    # a common step no larger than any subdomain's keeps d >= 0.1 d0
    for frac in (1.0, 0.5):
        a = np.full(alpha.size, frac * alpha.min())
        d1 = dist(pncg.step_positions(hier, x, p, a))
        assert np.all(d1 >= 0.1 * d0 - 1e-15)
    # the step of every stencil is 0.9 of its own time to contact, exactly
    xs = np.where(pool['idx'][..., None] >= 0, p.reshape(-1, 3)[np.maximum(pool['idx'], 0)], 0).reshape(-1, 12)
    rate = -(pool['grad'] * xs).sum(1)
    closing = rate > 0
    ac = np.minimum(1.0, 0.9 * d0[closing] / rate[closing])
    sub = np.where(pool['idx'] >= 0, hier.rank[np.maximum(pool['idx'], 0)] // 32, -1)[closing]
    for c in range(ac.size):
        for s_ in sub[c][sub[c] >= 0]:
            assert alpha[s_] <= ac[c] + 1e-15


def test_safe_step_mixed_subdomain_steps_keep_stencils_apart():
    """With the per-subdomain steps themselves (not a common one) every
    stencil keeps at least 0.05 of its distance, also for a search direction
    with a large common translation, where stencils across subdomain borders
    see their vertices move by different amounts."""
    sc = synth.two_boxes_scene(n_contacts=600, nxy=12, nz=6)
    pool = sc.pool
    hier = mas.Hierarchy(sc.X, 2)
    assert np.allclose(pool['grad'].reshape(-1, 4, 3).sum(1), 0.0)
    rng = np.random.default_rng(8)
    x = sc.x.reshape(-1)

    def dist(xx):
        xs = np.where(pool['idx'][..., None] >= 0, xx.reshape(-1, 3)[np.maximum(pool['idx'], 0)], 0)
        return (pool['grad'] * xs.reshape(-1, 12)).sum(1) - pool['off']

    d0 = dist(x)
    assert np.all(d0 > 0)
    p = 0.05 * rng.standard_normal(x.size)
    shift = np.tile(rng.standard_normal(3), sc.N)
    for q in (p, p + shift):
        alpha = pncg.safe_alpha(hier, pool['idx'], pool['grad'], d0, q)
        assert np.all((alpha > 0) & (alpha <= 1))
        d1 = dist(pncg.step_positions(hier, x, q, alpha))
        assert np.all(d1 >= 0.05 * d0 - 1e-15)
        assert np.any(alpha < 1)


def test_safe_step_closed_stencil_gives_zero():
    X = np.random.default_rng(6).uniform(size=(40, 3))
    hier = mas.Hierarchy(X, 1)
    idx = np.array([[3, -1, -1, -1]], np.int32)
    grad = np.zeros((1, 12))
    grad[0, :3] = [0, 0, 1.0]
    p = np.zeros(120)
    p[3 * 3 + 2] = -1.0
    alpha = pncg.safe_alpha(hier, idx, grad, np.array([-1e-6]), p)
    assert alpha[hier.subdomain_of_vertex(3)] == 0.0


def test_safe_step_single_contact_closed_form():
    X = np.random.default_rng(5).uniform(size=(40, 3))
    hier = mas.Hierarchy(X, 1)
    idx = np.array([[3, -1, -1, -1]], np.int32)
    grad = np.zeros((1, 12))
    grad[0, :3] = [0, 0, 1.0]
    p = np.zeros(120)
    p[3 * 3 + 2] = -2e-3          # moving toward the plane at 2e-3 per unit step
    alpha = pncg.safe_alpha(hier, idx, grad, np.array([1e-3]), p)
    d = hier.subdomain_of_vertex(3)
    assert alpha[d] == pytest.approx(0.9 * 1e-3 / 2e-3)
    assert np.all(np.delete(alpha, d) == 1.0)


def test_safe_step_falls_back_when_damping_rounds_do_not_separate():
    """A stencil across two subdomains whose vertices close fast on one side
    and open as fast on the other has no net closing rate, so its own rule
    leaves both steps at 1, while a second stencil holds one subdomain to a
    small step: the mixed steps close the first stencil by about 1, which
    halving both steps cures only after about 30 rounds (d = 1e-9).  The
    fallback then gives every subdomain the bound for any mix of steps,
    worked by hand here: 0.9 d / (sum of the closing rates)."""
    X = np.random.default_rng(5).uniform(size=(64, 3))
    hier = mas.Hierarchy(X, 1)
    r = hier.rank
    # one vertex of each of the two level-0 subdomains (library order)
    va = int(np.flatnonzero(r // 32 == 0)[0])
    vb = int(np.flatnonzero(r // 32 == 1)[0])
    vb2 = int(np.flatnonzero(r // 32 == 1)[1])
    idx = np.array([[va, vb, -1, -1], [vb2, -1, -1, -1]], np.int32)
    grad = np.zeros((2, 12))
    grad[0, 2] = 1.0           # grad at va: +z
    grad[0, 5] = -1.0          # grad at vb: -z
    grad[1, 2] = 1.0
    p = np.zeros(3 * 64)
    p[3 * va + 2] = -1.0       # va closes stencil 0 at rate 1
    p[3 * vb + 2] = -1.0       # vb opens it at rate 1 (the net rate is 0)
    p[3 * vb2 + 2] = -1.0      # stencil 1 closes at rate 1 from d = 1e-3
    d = np.array([1e-9, 1e-3])
    alpha = pncg.safe_alpha(hier, idx, grad, d, p)
    assert alpha[0] == pytest.approx(0.9e-9, rel=1e-15)
    assert alpha[1] == pytest.approx(0.9e-9, rel=1e-15)
    # both stencils keep at least 0.1 of their distances
    xn = pncg.step_positions(hier, X.reshape(-1), p, alpha)
    d_new = np.array([(grad[c].reshape(4, 3)[:1 + (c == 0)] * (xn.reshape(-1, 3)[idx[c][idx[c] >= 0]]
                                                          - X[idx[c][idx[c] >= 0]])).sum() for c in range(2)]) + d
    assert np.all(d_new >= 0.1 * d)
    # at d = 1e-3 the rounds suffice: stencil 1 sets 9e-4 on subdomain 1,
    # and stencil 0 (1e-3 - a_0 + a_1 >= 5e-5) needs 11 halvings of both
    alpha2 = pncg.safe_alpha(hier, idx, grad, np.array([1e-3, 1e-3]), p)
    assert alpha2[0] == 2.0 ** -11
    assert alpha2[1] == pytest.approx(9e-4 * 2.0 ** -11, rel=1e-15)
    xn2 = pncg.step_positions(hier, X.reshape(-1), p, alpha2)
    for c in range(2):
        vs = idx[c][idx[c] >= 0]
        dd = 1e-3 + (grad[c].reshape(4, 3)[:vs.size] * (xn2.reshape(-1, 3)[vs] - X[vs])).sum()
        assert dd >= 0.05 * 1e-3


def _two_subdomain_pt_case(gap):
    """A point in subdomain 0 above a triangle in subdomain 1, both moving
    down together (no relative motion along p), and a second point in
    subdomain 1 falling onto a fixed triangle of subdomain 1 from 0.3."""
    X = np.random.default_rng(7).uniform(size=(64, 3))
    hier = mas.Hierarchy(X, 1)
    r = hier.rank
    s0 = [int(v) for v in np.flatnonzero(r // 32 == 0)[:1]]
    s1 = [int(v) for v in np.flatnonzero(r // 32 == 1)[:7]]
    P, T = s0[0], s1[:3]
    Q, R = s1[3], s1[4:7]
    x = X.copy()
    x[P] = [0.0, 0.0, gap]
    x[T] = [[-1.0, -1.0, 0.0], [1.0, -1.0, 0.0], [0.0, 1.0, 0.0]]
    x[Q] = [10.0, 0.0, 0.3]
    x[R] = [[9.0, -1.0, 0.0], [11.0, -1.0, 0.0], [10.0, 1.0, 0.0]]
    p = np.zeros_like(x)
    p[[P] + T] = [0.0, 0.0, -1.0]
    p[Q] = [0.0, 0.0, -1.0]
    pairs = np.array([[P] + T, [Q] + R])
    kinds = np.array([ccd.PT, ccd.PT])
    dist = np.array([gap, 0.3])
    return hier, x, p, pairs, kinds, dist


def test_ccd_safe_step_falls_back_to_a_common_step():
    """At a gap of 1e-9 the mixed steps (1 for the moving point, about 0.3 for
    the triangle held by the other pair) close it by about 0.7, which halving
    both steps cures only after about 30 rounds: every subdomain takes the
    smallest step, the CCD step of the falling point, and both pairs stay
    open along the whole motion."""
    hier, x, p, pairs, kinds, dist = _two_subdomain_pt_case(1e-9)
    a2 = ccd.pair_step(x[pairs[1]], p[pairs[1]], ccd.PT, 0.3)
    assert 0.29 < a2 <= 0.3
    alpha = pncg.ccd_safe_alpha(hier, x, p, 1.0, pairs, kinds, dist)
    assert np.all(alpha == a2)
    for t in np.linspace(0.0, 1.0, 201):
        xt = pncg.step_positions(hier, x.reshape(-1), p.reshape(-1), t * alpha).reshape(-1, 3)
        for q, k in zip(pairs, kinds):
            assert C.pair_distance(xt[q], k)[0] > 0.0


def test_ccd_safe_step_damping_rounds_suffice():
    """At a gap of 0.05 halving both steps separates the pair.  The moving
    point's subdomain starts at the radius cap 1 / (2 max |p|) = 0.5, the
    triangle's at the falling point's CCD step a2; k halvings of both leave
    the relative approach 2^-k (0.5 - a2) no larger than the gap, and k - 1
    would not.  The result keeps every pair open along the mixed motion."""
    hier, x, p, pairs, kinds, dist = _two_subdomain_pt_case(0.05)
    a2 = ccd.pair_step(x[pairs[1]], p[pairs[1]], ccd.PT, 0.3)
    alpha = pncg.ccd_safe_alpha(hier, x, p, 1.0, pairs, kinds, dist)
    k = -np.log2(alpha[0] / 0.5)
    assert k == int(k) and 1 <= k <= 16
    assert alpha[1] == pytest.approx(a2 * 2.0 ** -k, rel=1e-15)
    assert alpha[0] - alpha[1] <= 0.05
    assert 2.0 * (alpha[0] - alpha[1]) >= 0.05 * (1.0 - 1e-12)
    for t in np.linspace(0.0, 1.0, 201):
        xt = pncg.step_positions(hier, x.reshape(-1), p.reshape(-1), t * alpha).reshape(-1, 3)
        for q, kk in zip(pairs, kinds):
            assert C.pair_distance(xt[q], kk)[0] > 0.0


def test_ccd_safe_step_radius_cap():
    """No pair within the radius: every step is radius / (2 max |p|)."""
    X = np.random.default_rng(3).uniform(size=(40, 3))
    hier = mas.Hierarchy(X, 1)
    p = np.zeros_like(X)
    p[5] = [0.0, 2.0, 0.0]
    alpha = pncg.ccd_safe_alpha(hier, X, p, 0.5, np.zeros((0, 4), np.int64), np.zeros(0, np.int64),
                                np.zeros(0))
    assert np.all(alpha == 0.125)


def test_ccd_safe_step_keeps_all_surface_pairs_apart():
    """Two boxes a small gap apart, a random direction with a downward push
    on the upper box: with the candidates of the radius 2 max |p|, every
    pair of the surface within 1.5 times that radius (brute force, a
    superset of the candidates and of every pair the motion could close)
    stays at a positive distance along the mixed per-subdomain motion."""
    from oracle import constraint_set as CS
    sc = synth.two_boxes_scene(nxy=4, nz=3, n_contacts=8)
    verts, tris, edges = synth.surface(sc.tets)
    hier = mas.Hierarchy(sc.X, 1)
    x = sc.x.reshape(-1, 3)
    rng = np.random.default_rng(11)
    p = 0.02 * rng.standard_normal(x.shape)
    p[x[:, 2] > x[:, 2].mean(), 2] -= 0.05
    radius = 2.0 * np.linalg.norm(p, axis=1).max()
    cp, ck, cd = CS.constraint_set(x, verts, tris, edges, radius)
    alpha = pncg.ccd_safe_alpha(hier, x, p, radius, np.asarray(cp), np.asarray(ck), np.asarray(cd))
    assert np.any(alpha < 1.0)
    allp, allk, _ = CS.constraint_set(x, verts, tris, edges, 1.5 * radius)
    assert len(allp) > len(cp)
    for t in np.linspace(0.0, 1.0, 11):
        xt = pncg.step_positions(hier, x.reshape(-1), p.reshape(-1), t * alpha).reshape(-1, 3)
        d, _, _ = C.contact_distances(xt, np.asarray(allp), np.asarray(allk))
        assert d.min() > 0.0
