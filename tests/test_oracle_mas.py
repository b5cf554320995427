"""Pins of the oracle's Morton hierarchy and MAS preconditioner.

Anchors: hand-derived Morton codes, the reduction of MAS to an exact
inverse when one subdomain covers the mesh or when the matrix has no
coupling between subdomains, closed-form coarse matrices for the identity
operator, the energy identity of the Galerkin projection, and symmetry /
positive definiteness of P on the small grid scene.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, mas
from paper_2604_19892_amd import synth


def test_morton_codes_hand_derived():
    # corners of the unit cube after normalisation to the bounding box
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [0.5, 0.5, 0.5]], float)
    c = mas.morton_codes(X)
    full = (1 << 21) - 1
    # x bits occupy positions 0,3,6,..; y bits 1,4,..; z bits 2,5,..
    xbits = sum(1 << (3 * b) for b in range(21))
    assert int(c[0]) == 0
    assert int(c[1]) == xbits
    assert int(c[2]) == xbits << 1
    assert int(c[3]) == xbits << 2
    assert int(c[4]) == (1 << 63) - 1
    # 0.5 * (2^21 - 1) floors to 2^20 - 1: every bit but the top one
    half = (1 << 20) - 1
    assert int(c[5]) == sum(7 << (3 * b) for b in range(20))
    assert full == 2097151 and half == 1048575


def test_morton_order_is_z_curve_on_2x2x2():
    X = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], float)
    perm = mas.morton_perm(X[::-1].copy())
    # reversed input: the Z-curve visits x fastest, then y, then z
    np.testing.assert_array_equal(perm, np.arange(8)[::-1])


def test_morton_ties_keep_original_order():
    X = np.array([[0, 0, 0], [1, 1, 1], [0, 0, 0], [1, 1, 1]], float)
    np.testing.assert_array_equal(mas.morton_perm(X), [0, 2, 1, 3])


def spd(rng, n):
    A = rng.standard_normal((n, n))
    return A @ A.T + n * np.eye(n)


def test_single_subdomain_single_level_is_exact_inverse():
    rng = np.random.default_rng(0)
    X = rng.uniform(size=(20, 3))
    hier = mas.Hierarchy(X, levels=1)
    A = spd(rng, 60)
    P = mas.MAS(hier, sp.csr_matrix(A))
    g = rng.standard_normal(60)
    np.testing.assert_allclose(P.apply(g), np.linalg.solve(A, g), rtol=1e-12)


def test_block_diagonal_matrix_level0_is_exact():
    rng = np.random.default_rng(1)
    X = rng.uniform(size=(100, 3))
    hier = mas.Hierarchy(X, levels=1)
    A = np.zeros((300, 300))
    for d in range(hier.num_subdomains()):
        dofs = hier.subdomain_dofs(d)
        A[np.ix_(dofs, dofs)] = spd(rng, dofs.size)
    P = mas.MAS(hier, sp.csr_matrix(A))
    g = rng.standard_normal(300)
    np.testing.assert_allclose(P.apply(g), np.linalg.solve(A, g), rtol=1e-11)


def test_coarse_matrices_of_identity_are_member_counts():
    rng = np.random.default_rng(2)
    N = 1000
    X = rng.uniform(size=(N, 3))
    hier = mas.Hierarchy(X, levels=3)
    P = mas.MAS(hier, sp.identity(3 * N, format='csr'))
    # level l node a holds min(32^l, N - 32^l a) vertices
    for l, (Cl, Al, invs) in enumerate(P.coarse, start=1):
        n_nodes = hier.num_nodes(l)
        cnt = np.array([min(32 ** l, N - 32 ** l * a) for a in range(n_nodes)], float)
        np.testing.assert_allclose(Al.toarray(), np.diag(np.repeat(cnt, 3)))
    # and P applied to a constant vector: level 0 gives 1, each level adds 1
    z = P.apply(np.ones(3 * N))
    np.testing.assert_allclose(z, 3.0)


def test_galerkin_energy_identity(grid):
    prob = fem.Problem(grid)
    base, _ = synth.grid_update_sets(grid)
    H = prob.assemble(grid.x, base)
    hier = mas.Hierarchy(grid.X, levels=2)
    Cl = hier.C(1)
    Al = Cl @ H @ Cl.T
    rng = np.random.default_rng(3)
    y = rng.standard_normal(Al.shape[0])
    e = Cl.T @ y          # prolongation: every vertex of node a takes y_a
    np.testing.assert_allclose(y @ (Al @ y), e @ (H @ e), rtol=1e-12)
    # the prolongated vector is constant over each node's vertices
    node = hier.rank // 32
    E = e.reshape(-1, 3)
    for a in range(hier.num_nodes(1)):
        np.testing.assert_allclose(E[node == a], np.repeat(y[3 * a:3 * a + 3][None], (node == a).sum(), 0))


def test_preconditioner_symmetric_positive_definite(grid):
    prob = fem.Problem(grid)
    base, _ = synth.grid_update_sets(grid)
    H = prob.assemble(grid.x, base)
    hier = mas.Hierarchy(grid.X, levels=2)
    P = mas.MAS(hier, H).dense()
    np.testing.assert_allclose(P, P.T, rtol=0, atol=1e-13 * np.abs(P).max())
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0
    # level 0 alone restricted to a subdomain inverts that block
    for d in (0, 7, 15):
        dofs = hier.subdomain_dofs(d)
        B = mas.MAS(hier, H).fine[d]
        np.testing.assert_allclose(B @ H[dofs][:, dofs].toarray(), np.eye(dofs.size), atol=1e-9)


def test_subdomain_sizes_for_paper_shaped_counts():
    hier = mas.Hierarchy(np.random.default_rng(0).uniform(size=(1140096, 3))[:10], levels=4)
    # the counting rule D_l = ceil(N_l / 32), N_{l+1} = D_l
    h = mas.Hierarchy.__new__(mas.Hierarchy)
    h.N = 1140096
    assert [h.num_subdomains(l) for l in range(4)] == [35628, 1114, 35, 2]
    h.N = 64000
    assert [h.num_subdomains(l) for l in range(3)] == [2000, 63, 2]
    assert hier.N == 10
