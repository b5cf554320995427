"""Pins of the 3x3 block-Jacobi oracle: hand-inverted blocks, the exact
inverse of a block-diagonal matrix, and independence from the couplings
between vertices."""
import numpy as np
import scipy.sparse as sp

from oracle import jacobi


def test_hand_blocks():
    # vertex 0: diag(2, 4, 8); vertex 1: [[2, 1, 0], [1, 2, 0], [0, 0, 1]],
    # whose inverse is [[2, -1, 0], [-1, 2, 0], [0, 0, 3]] / 3
    H = np.zeros((6, 6))
    H[:3, :3] = np.diag([2.0, 4.0, 8.0])
    H[3:, 3:] = [[2.0, 1.0, 0.0], [1.0, 2.0, 0.0], [0.0, 0.0, 1.0]]
    inv = jacobi.inverse_blocks(H)
    np.testing.assert_allclose(inv[0], np.diag([0.5, 0.25, 0.125]), rtol=1e-15)
    np.testing.assert_allclose(inv[1], np.array([[2.0, -1.0, 0.0], [-1.0, 2.0, 0.0], [0.0, 0.0, 3.0]]) / 3.0,
                               rtol=1e-15, atol=1e-16)
    z = jacobi.apply(inv, [2.0, 4.0, 8.0, 3.0, 0.0, 3.0])
    np.testing.assert_allclose(z, [1.0, 1.0, 1.0, 2.0, -1.0, 3.0], rtol=1e-15, atol=1e-15)


def test_block_diagonal_matrix_is_inverted_exactly():
    rng = np.random.default_rng(0)
    n = 7
    blocks = []
    for _ in range(n):
        A = rng.standard_normal((3, 3))
        blocks.append(A @ A.T + 0.5 * np.eye(3))
    H = sp.block_diag(blocks).tocsr()
    inv = jacobi.inverse_blocks(H)
    g = rng.standard_normal(3 * n)
    z = jacobi.apply(inv, g)
    np.testing.assert_allclose(H @ z, g, rtol=1e-12, atol=1e-12)


def test_couplings_between_vertices_are_ignored():
    rng = np.random.default_rng(1)
    n = 5
    A = rng.standard_normal((3 * n, 3 * n))
    H = A @ A.T + 3 * n * np.eye(3 * n)
    D = np.zeros_like(H)
    for i in range(n):
        D[3 * i:3 * i + 3, 3 * i:3 * i + 3] = H[3 * i:3 * i + 3, 3 * i:3 * i + 3]
    g = rng.standard_normal(3 * n)
    np.testing.assert_allclose(jacobi.apply(jacobi.inverse_blocks(H), g), np.linalg.solve(D, g), rtol=1e-12)
    # symmetric positive definite preconditioner
    P = np.column_stack([jacobi.apply(jacobi.inverse_blocks(H), e) for e in np.eye(3 * n)])
    np.testing.assert_allclose(P, P.T, atol=1e-14)
    assert np.linalg.eigvalsh(P).min() > 0
