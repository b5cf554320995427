"""Pins of the comparison direction rules (FR, CD, DK) and of the loop
variants of the ablations (update strategy, direction rule), against
mathematics they must satisfy:

* hand-worked beta values on a two-dimensional case;
* on a strictly convex quadratic with exact steps every rule, and the 2x2
  subspace step, is preconditioned linear CG: A-conjugate directions,
  P-orthogonal gradients and the exact minimiser after n steps;
* CD and DK are invariant to the scale of the previous direction (beta
  scales inversely), FR is not;
* the safeguards: a non-positive denominator or an ascent direction gives
  d = -z with the fallback flag.
"""
import numpy as np
import pytest

from oracle import pncg

RULES = (pncg.BETA_FR, pncg.BETA_CD, pncg.BETA_DK)


def test_hand_values():
    # g = (1, 2), g_prev = (3, 1), P = I, d_prev = (-1, 0):
    # FR = 5 / 10; CD = 5 / 3; DK: y = (-2, 1), d.y = 2, y.z = 0, y.Py = 5,
    # d.g = -1, so beta = 0 - (5 / 2)(-1 / 2) = 1.25
    g, gp, dp = np.array([1.0, 2.0]), np.array([3.0, 1.0]), np.array([-1.0, 0.0])
    assert pncg.beta_coefficient(pncg.BETA_FR, g, gp, g, gp, dp) == pytest.approx(0.5, rel=1e-15)
    assert pncg.beta_coefficient(pncg.BETA_CD, g, gp, g, gp, dp) == pytest.approx(5.0 / 3.0, rel=1e-15)
    assert pncg.beta_coefficient(pncg.BETA_DK, g, gp, g, gp, dp) == pytest.approx(1.25, rel=1e-15)
    # FR step with H~ = I: d = (-1.5, -2), g.d = -5.5, d.d = 6.25
    a, b, d, p, fb = pncg.beta_step(pncg.BETA_FR, g, gp, g, gp, dp, lambda v: v, False)
    assert not fb and b == 0.5
    np.testing.assert_allclose(d, [-1.5, -2.0], rtol=0, atol=0)
    assert a == pytest.approx(5.5 / 6.25, rel=1e-15)
    np.testing.assert_allclose(p, a * d, rtol=1e-15)


def _quadratic(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.geomspace(1.0, 20.0, n)) @ Q.T
    A = 0.5 * (A + A.T)
    R = rng.standard_normal((n, n))
    P = np.linalg.inv(np.diag(np.diag(A))) + 0.05 * (R @ R.T) / n   # SPD, not A^-1
    b = rng.standard_normal(n)
    return A, P, b, rng.standard_normal(n)


@pytest.mark.parametrize("rule", RULES + ("subspace",))
def test_quadratic_is_preconditioned_cg(rule):
    n = 8
    A, P, b, x = _quadratic(n, 11)
    xs = np.linalg.solve(A, b)
    restart, g_prev, z_prev, d_prev, p = True, None, None, None, np.zeros(n)
    ds, gs = [], []
    for k in range(n):
        g = A @ x - b
        z = P @ g
        gs.append(g)
        if rule == "subspace":
            mu, nu, p, fb, *_ = pncg.subspace_step(g, z, p, lambda v: A @ v, restart)
            d = p
        else:
            a, beta, d, p, fb = pncg.beta_step(rule, g, g_prev, z, z_prev, d_prev, lambda v: A @ v, restart)
        assert not fb
        ds.append(d)
        x = x + p
        restart, g_prev, z_prev, d_prev = False, g, z, d
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    D = np.array(ds)
    G = np.array(gs)
    C = D @ A @ D.T
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() <= 1e-9 * np.abs(np.diag(C)).max()
    Gp = G @ P @ G.T
    offg = Gp - np.diag(np.diag(Gp))
    assert np.abs(offg).max() <= 1e-9 * np.abs(np.diag(Gp)).max()


def test_scale_of_previous_direction():
    rng = np.random.default_rng(2)
    for _ in range(50):
        g, gp, z, zp, dp = rng.standard_normal((5, 6))
        for rule, covariant in ((pncg.BETA_CD, True), (pncg.BETA_DK, True), (pncg.BETA_FR, False)):
            b1 = pncg.beta_coefficient(rule, g, gp, z, zp, dp)
            b2 = pncg.beta_coefficient(rule, g, gp, z, zp, 3.0 * dp)
            if b1 is None:
                assert b2 is None
                continue
            if covariant:
                assert b2 * 3.0 == pytest.approx(b1, rel=1e-12)
            else:
                assert b2 == b1


def test_safeguards():
    g = np.array([1.0, 0.0])
    z = g.copy()
    # FR with g_prev^T z_prev = 0: no beta
    a, b, d, p, fb = pncg.beta_step(pncg.BETA_FR, g, np.zeros(2), z, np.zeros(2), np.array([1.0, 1.0]),
                                    lambda v: v, False)
    assert fb and b == 0.0
    np.testing.assert_array_equal(d, -z)
    # CD with an ascent previous direction (d_prev^T g_prev > 0): no beta
    a, b, d, p, fb = pncg.beta_step(pncg.BETA_CD, g, np.array([0.0, 1.0]), z, np.array([0.0, 1.0]),
                                    np.array([0.0, 1.0]), lambda v: v, False)
    assert fb and b == 0.0
    # FR whose beta d_prev turns d uphill: g = (1, 0), beta = 1 / 0.25 = 4,
    # d_prev = (1, 0) gives d = (3, 0), g.d = 3 > 0
    a, b, d, p, fb = pncg.beta_step(pncg.BETA_FR, g, np.array([0.5, 0.0]), z, np.array([0.5, 0.0]),
                                    np.array([1.0, 0.0]), lambda v: v, False)
    assert fb and b == 0.0
    np.testing.assert_array_equal(d, -z)
    assert a == pytest.approx(1.0)
    # non-positive curvature: alpha = 1
    a, b, d, p, fb = pncg.beta_step(pncg.BETA_FR, g, None, z, None, None, lambda v: -v, True)
    assert fb and a == 1.0
    # the restart form equals the subspace step's
    A = np.diag([2.0, 3.0])
    a, b, d, p, fb = pncg.beta_step(pncg.BETA_DK, g, None, z, None, None, lambda v: A @ v, True)
    mu, nu, p2, fb2, *_ = pncg.subspace_step(g, z, None, lambda v: A @ v, True)
    assert not fb and not fb2 and a == mu and np.array_equal(p, p2)


# ------------------------------------------------------------ loop variants
# The ablation loops compose pinned steps; these check the composition.

@pytest.fixture(scope="module")
def grid():
    from paper_2604_19892_amd import synth
    return synth.grid_scene()


def test_variants_share_the_restart_iteration(grid):
    from oracle import solver
    ref = None
    for update in ("woodbury", "freeze", "rebuild"):
        for rule in ("subspace", "fr", "cd", "dk"):
            s = solver.OraclePNCG(grid, update=update, rule=rule)
            g, z, p = s.iterate()
            if ref is None:
                ref = p
            np.testing.assert_allclose(p, ref, rtol=0, atol=1e-14 * np.abs(ref).max())


def test_freeze_keeps_the_restart_preconditioner(grid):
    from oracle import solver
    s = solver.OraclePNCG(grid, update="freeze")
    s.iterate()
    assert not s.restart
    fine = [b.copy() for b in s.mas.fine]
    g, z, p = s.iterate()
    assert not s.log[-1]['restart']
    np.testing.assert_allclose(z, s.mas.apply(g, fine), rtol=1e-13, atol=0)
    # the Woodbury strategy's preconditioner differs once contacts changed
    w = solver.OraclePNCG(grid, update="woodbury")
    w.iterate()
    gw, zw, _ = w.iterate()
    assert np.array_equal(gw, g)
    assert np.linalg.norm(zw - z) > 1e-8 * np.linalg.norm(z)


def test_rebuild_reassembles_at_every_iterate(grid):
    from oracle import fem, solver
    s = solver.OraclePNCG(grid, update="rebuild")
    s.iterate()
    x1 = s.x.copy()
    s.iterate()
    assert not s.log[-1]['restart']
    C = s.constraint_set(x1)
    H = fem.Problem(grid).assemble(x1, C)
    assert abs(s.H_base - H).max() <= 1e-12 * abs(H).max()
    assert np.array_equal(s.base['key'], C['key'])


@pytest.mark.parametrize("update,rule", [("freeze", "subspace"), ("rebuild", "subspace"), ("woodbury", "fr"),
                                         ("woodbury", "cd"), ("woodbury", "dk")])
def test_variants_never_raise_the_energy(grid, update, rule):
    from oracle import solver
    s = solver.OraclePNCG(grid, update=update, rule=rule)
    for _ in range(4):
        s.iterate()
    E = [r['E'] for r in s.log] + [s.prob.energy(s.x, s.x_tilde, s.constraint_set(s.x))]
    assert all(b <= a for a, b in zip(E, E[1:]))
    assert E[-1] < E[0]


def test_block_jacobi_loop(grid):
    from oracle import fem, jacobi, solver
    s = solver.OraclePNCG(grid, precond="bj3")
    x0 = s.x.copy()
    C = s.constraint_set(x0)
    g, z, p = s.iterate()
    H = fem.Problem(grid).assemble(x0, C)
    np.testing.assert_allclose(z, jacobi.apply(jacobi.inverse_blocks(H), g), rtol=1e-13, atol=0)
    for _ in range(3):
        s.iterate()
    E = [r['E'] for r in s.log]
    assert all(b <= a for a, b in zip(E, E[1:])) and E[-1] < E[0]
