"""Pins of the oracle's energy, gradient and Hessian snapshot.

Each check is anchored outside the oracle's own formulas: closed forms,
invariants of the stable Neo-Hookean energy, central finite differences,
and exact properties of affine (rank-one) contact stencils.
"""
import numpy as np
import pytest

from oracle import fem
from paper_2604_19892_amd import synth


def rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# ----------------------------------------------------------------- barrier

def test_barrier_closed_form_values():
    dhat = 1e-3
    d = np.array([1e-5, 5e-4, dhat, 2 * dhat])
    b, b1, b2 = fem.barrier(d, dhat)
    # b(d) = -(d - dhat)^2 ln(d/dhat); hand-evaluated at d = dhat/2
    assert b[1] == pytest.approx(-(0.5e-3) ** 2 * np.log(0.5), rel=1e-14)
    # vanishes with its first two derivatives at dhat and beyond
    assert b[2] == 0 and b1[2] == 0 and b2[2] == 0
    assert b[3] == 0 and b1[3] == 0 and b2[3] == 0
    # b'' at 1e-5: -2 ln(0.01) + 4*99 + 99^2 (hand expansion)
    assert b2[0] == pytest.approx(-2 * np.log(0.01) + 4 * 99 + 99 ** 2, rel=1e-12)


def test_barrier_derivatives_by_finite_differences():
    dhat = 1e-3
    d = np.geomspace(2e-6, 0.9e-3, 25)
    eps = d * 1e-6
    b, b1, b2 = fem.barrier(d, dhat)
    bp, b1p, _ = fem.barrier(d + eps, dhat)
    bm, b1m, _ = fem.barrier(d - eps, dhat)
    np.testing.assert_allclose((bp - bm) / (2 * eps), b1, rtol=1e-6)
    np.testing.assert_allclose((b1p - b1m) / (2 * eps), b2, rtol=1e-6)
    assert np.all(b2 > 0) and np.all(b1 < 0) and np.all(b > 0)


# ------------------------------------------------------------ elasticity

def test_snh_rest_and_rotation_invariance():
    rng = np.random.default_rng(3)
    mu, lam = fem.lame(np.full(5, 1e5), np.full(5, 0.4))
    I = np.repeat(np.eye(3)[None], 5, 0)
    assert np.allclose(fem.snh_psi(I, mu, lam), 0.0)
    assert np.allclose(fem.snh_P(I, mu, lam), 0.0)
    F = np.eye(3)[None] + 0.2 * rng.standard_normal((5, 3, 3))
    R = np.stack([rot(rng) for _ in range(5)])
    np.testing.assert_allclose(fem.snh_psi(R @ F, mu, lam), fem.snh_psi(F, mu, lam), rtol=1e-11)


def test_lame_closed_form():
    mu, lam = fem.lame(1e5, 0.4)
    assert float(mu) == pytest.approx(35714.285714285714, rel=1e-14)
    assert float(lam) == pytest.approx(142857.14285714287, rel=1e-14)


def test_snh_stress_and_tangent_by_finite_differences():
    rng = np.random.default_rng(4)
    T = 4
    mu, lam = fem.lame(np.full(T, 1e5), np.full(T, 0.4))
    F = np.eye(3)[None] + 0.3 * rng.standard_normal((T, 3, 3))
    P = fem.snh_P(F, mu, lam)
    H = fem.snh_dPdF(F, mu, lam)
    eps = 1e-6
    for a in range(3):
        for b in range(3):
            dF = np.zeros((T, 3, 3))
            dF[:, a, b] = eps
            dpsi = (fem.snh_psi(F + dF, mu, lam) - fem.snh_psi(F - dF, mu, lam)) / (2 * eps)
            np.testing.assert_allclose(dpsi, P[:, a, b], rtol=1e-6, atol=1e-3)
            dP = (fem.vecF(fem.snh_P(F + dF, mu, lam)) - fem.vecF(fem.snh_P(F - dF, mu, lam))) / (2 * eps)
            np.testing.assert_allclose(dP, H[:, :, 3 * b + a], rtol=1e-6, atol=1e-2)


def test_rest_quantities_of_unit_cube(grid):
    Dm_inv, vol, mass = fem.rest_quantities(grid.X, grid.tets, grid.density)
    assert vol.sum() == pytest.approx(1.0, rel=1e-12)        # unit cube
    assert mass.sum() == pytest.approx(1000.0, rel=1e-12)    # rho * volume
    assert np.all(vol > 0)
    P = grid.X[grid.tets]
    Dm = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    np.testing.assert_allclose(Dm_inv @ Dm, np.repeat(np.eye(3)[None], len(vol), 0), atol=1e-12)


def test_gradient_by_finite_differences(grid):
    prob = fem.Problem(grid)
    rng = np.random.default_rng(5)
    cset = synth.grid_update_sets(grid)[0]
    xt = fem.inertial_target(grid.x, grid.v, grid.h, grid.gravity).reshape(-1)
    x = grid.x.reshape(-1).copy()
    # contacts: point-plane stencils are affine, d(x) changes with x
    pool = grid.pool

    def dist(xx):
        return (pool['grad'] * fem.stencil_gather(pool['idx'], xx)).sum(1) - pool['off']

    def E(xx):
        c = dict(cset)
        c['d'] = dist(xx)
        return prob.energy(xx, xt, c)

    c0 = dict(cset)
    c0['d'] = dist(x)
    g = prob.gradient(x, xt, c0)
    dirs = rng.standard_normal((6, x.size))
    for v in dirs:
        h = 2e-7                    # fourth-order central difference
        fd = (-E(x + 2 * h * v) + 8 * E(x + h * v) - 8 * E(x - h * v) + E(x - 2 * h * v)) / (12 * h)
        assert fd == pytest.approx(float(g @ v), rel=1e-7, abs=1e-9)


def test_unprojected_hessian_by_finite_differences_of_gradient(grid):
    prob = fem.Problem(grid)
    x = grid.x.copy()
    He = prob.elastic_hessians(x, project=False)
    rng = np.random.default_rng(6)
    tets = prob.tets[:20]
    for t in range(20):
        v = rng.standard_normal(12)
        eps = 1e-6
        xp = x.copy()
        xm = x.copy()
        xp[tets[t]] += eps * v.reshape(4, 3)
        xm[tets[t]] -= eps * v.reshape(4, 3)
        sl = slice(t, t + 1)
        gp = fem.elastic_gradient(xp, tets[sl], prob.Dm_inv[sl], prob.vol[sl], prob.mu[sl], prob.lam[sl])
        gm = fem.elastic_gradient(xm, tets[sl], prob.Dm_inv[sl], prob.vol[sl], prob.mu[sl], prob.lam[sl])
        fd = ((gp - gm) / (2 * eps))[tets[t]].reshape(-1) * prob.h ** 2
        np.testing.assert_allclose(He[t] @ v, fd, rtol=1e-5, atol=1e-9 * np.abs(fd).max())


def test_projection_is_psd_and_idempotent_on_psd():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((10, 9, 9))
    S = A + np.transpose(A, (0, 2, 1))
    P = fem.psd_project(S)
    assert np.all(np.linalg.eigvalsh(P) > -1e-12)
    # a PSD input is returned unchanged
    Q = A @ np.transpose(A, (0, 2, 1))
    np.testing.assert_allclose(fem.psd_project(Q), Q, rtol=1e-10, atol=1e-10)
    # the projection removes exactly the negative part: S = P - N, N PSD, P N = 0
    Nn = P - S
    assert np.all(np.linalg.eigvalsh(Nn) > -1e-10)
    np.testing.assert_allclose(P @ Nn, 0.0, atol=1e-9)


def test_projected_element_hessians_psd_and_match_when_psd(grid):
    prob = fem.Problem(grid)
    Hp = prob.elastic_hessians(grid.x, project=True)
    Hu = prob.elastic_hessians(grid.x, project=False)
    ev = np.linalg.eigvalsh(Hp)
    assert np.all(ev > -1e-12 * np.abs(ev).max())
    psd = np.linalg.eigvalsh(Hu).min(1) > 0
    np.testing.assert_allclose(Hp[psd], Hu[psd], rtol=1e-9, atol=1e-12)
    # rigid motions (translations) are in the null space of every element Hessian
    t = np.tile(np.array([1.0, -2.0, 0.5]), 4)
    assert np.abs(Hp @ t).max() < 1e-9 * np.abs(Hp).max()


def test_affine_contact_hessian_is_exactly_rank_one():
    """For d affine in x the barrier Hessian is kappa b''(d) n n^T exactly,
    so the contact part of H_base equals finite differences of the
    contact gradient."""
    sc = synth.two_boxes_scene(n_contacts=200, nxy=6, nz=4)
    prob = fem.Problem(sc)
    pool = sc.pool
    x = sc.x.reshape(-1)

    def cgrad(xx):
        d = (pool['grad'] * fem.stencil_gather(pool['idx'], xx)).sum(1) - pool['off']
        _, b1, _ = fem.barrier(d, prob.dhat)
        return fem.stencil_scatter(pool['idx'], (prob.kappa * b1)[:, None] * pool['grad'], prob.N).reshape(-1)

    d0 = (pool['grad'] * fem.stencil_gather(pool['idx'], x)).sum(1) - pool['off']
    Hc = fem.contact_outer(pool['idx'], pool['grad'], prob.contact_stiffness(d0), prob.N)
    rng = np.random.default_rng(8)
    for _ in range(3):
        v = rng.standard_normal(x.size)
        eps = 1e-11
        fd = (cgrad(x + eps * v) - cgrad(x - eps * v)) / (2 * eps)
        np.testing.assert_allclose(Hc @ v, fd, rtol=1e-4, atol=1e-6 * np.abs(fd).max())


def test_assembled_hessian_symmetric_spd(grid):
    prob = fem.Problem(grid)
    base, _ = synth.grid_update_sets(grid)
    H = prob.assemble(grid.x, base).toarray()
    np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-12 * np.abs(H).max())
    assert np.linalg.eigvalsh(H).min() > 0
    # constant translations: only the mass and the contacts act on them
    t = np.tile([1.0, 0, 0], prob.N)
    Hel = H - np.diag(np.repeat(prob.mass, 3)) - fem.contact_outer(
        base['idx'], base['grad'], prob.contact_stiffness(base['d']), prob.N).toarray()
    assert np.abs(Hel @ t).max() < 1e-10 * np.abs(Hel).max()
