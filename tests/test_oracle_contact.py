"""Pins of the contact-distance oracle (point-triangle and edge-edge
distance, closest-feature type and the envelope gradient n = grad d of
Section 4.1) against closed forms, brute-force sampling, finite
differences and invariances."""
import numpy as np
import pytest

from oracle import contact as C


def rot(rng):
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    return q * np.sign(np.linalg.det(q))


TRI = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])


def test_point_above_face():
    h = 0.37
    d, g, ty = C.pair_distance(np.vstack([[0.2, 0.3, h], TRI]), C.PT)
    assert d == pytest.approx(h, abs=1e-15) and ty == 6
    n = np.array([0.0, 0.0, 1.0])
    w = np.array([0.5, 0.2, 0.3])
    want = np.concatenate([n, -w[0] * n, -w[1] * n, -w[2] * n])
    assert np.allclose(g, want, atol=1e-14)


def test_point_vertex_and_edge_regions():
    d, _, ty = C.pair_distance(np.vstack([[-1.0, -1.0, 0.5], TRI]), C.PT)
    assert d == pytest.approx(np.sqrt(2.25), abs=1e-15) and ty == 0
    d, _, ty = C.pair_distance(np.vstack([[0.5, -1.0, 0.0], TRI]), C.PT)
    assert d == pytest.approx(1.0, abs=1e-15) and ty == 3
    d, _, ty = C.pair_distance(np.vstack([[1.0, 1.0, 0.0], TRI]), C.PT)  # beyond the hypotenuse
    assert d == pytest.approx(np.sqrt(0.5), abs=1e-15) and ty == 4
    d, _, ty = C.pair_distance(np.vstack([[2.0, -0.5, 0.0], TRI]), C.PT)  # beyond T1
    assert d == pytest.approx(np.sqrt(1.25), abs=1e-15) and ty == 1


def test_crossing_edges():
    h = 0.25
    X = np.array([[-1.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, -1.0, h], [0.0, 1.0, h]])
    d, g, ty = C.pair_distance(X, C.EE)
    assert d == pytest.approx(h, abs=1e-15) and ty == 8
    n = np.array([0.0, 0.0, -1.0])
    assert np.allclose(g, np.concatenate([0.5 * n, 0.5 * n, -0.5 * n, -0.5 * n]), atol=1e-14)


def test_parallel_and_degenerate_edges():
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, 1.0, 0.0], [1.5, 1.0, 0.0]])
    assert C.pair_distance(X, C.EE)[0] == pytest.approx(1.0, abs=1e-15)
    # a zero-length edge is a point: point-segment distance
    X = np.array([[0.3, 2.0, 0.0], [0.3, 2.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    assert C.pair_distance(X, C.EE)[0] == pytest.approx(2.0, abs=1e-15)
    # collinear triangle: distance to its longest side
    T = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    d, _, _ = C.pair_distance(np.vstack([[1.5, 0.7, 0.0], T]), C.PT)
    assert d == pytest.approx(0.7, abs=1e-15)
    # a point on the triangle: zero distance, zero gradient
    d, g, _ = C.pair_distance(np.vstack([[0.25, 0.25, 0.0], TRI]), C.PT)
    assert d == 0.0 and not g.any()


def _sample_min(X, kind, n=160):
    u = np.linspace(0.0, 1.0, n + 1)
    if kind == C.PT:
        U, V = np.meshgrid(u, u, indexing="ij")
        keep = U + V <= 1.0 + 1e-15
        U, V = U[keep], V[keep]
        P = X[1] + U[:, None] * (X[2] - X[1]) + V[:, None] * (X[3] - X[1])
        return np.linalg.norm(P - X[0], axis=1).min(), np.linalg.norm(X[1:] - X[[2, 3, 1]], axis=1).max() / n
    S, T = np.meshgrid(u, u, indexing="ij")
    A = X[0] + S.reshape(-1, 1) * (X[1] - X[0])
    B = X[2] + T.reshape(-1, 1) * (X[3] - X[2])
    span = np.linalg.norm(X[1] - X[0]) + np.linalg.norm(X[3] - X[2])
    return np.linalg.norm(A - B, axis=1).min(), span / n


@pytest.mark.parametrize("kind", [C.PT, C.EE])
def test_brute_force_sampling(kind):
    rng = np.random.default_rng(7 + kind)
    for _ in range(40):
        X = rng.standard_normal((4, 3))
        d = C.pair_distance(X, kind)[0]
        smin, h = _sample_min(X, kind)
        # no sample is closer than the minimum; some sample is within the grid spacing of it
        assert smin >= d - 1e-12
        assert smin <= d + 2.0 * h


@pytest.mark.parametrize("kind", [C.PT, C.EE])
def test_gradient_finite_differences(kind):
    rng = np.random.default_rng(11 + kind)
    checked = 0
    for _ in range(40):
        X = rng.standard_normal((4, 3))
        d, g, _ = C.pair_distance(X, kind)
        if d < 1e-3:
            continue
        eps = 1e-6
        fd = np.zeros(12)
        for q in range(12):
            Xp, Xm = X.copy(), X.copy()
            Xp.flat[q] += eps
            Xm.flat[q] -= eps
            fd[q] = (C.pair_distance(Xp, kind)[0] - C.pair_distance(Xm, kind)[0]) / (2 * eps)
        assert np.allclose(g, fd, atol=1e-6), (g, fd)
        checked += 1
    assert checked > 30


@pytest.mark.parametrize("kind", [C.PT, C.EE])
def test_rigid_motion_and_permutation(kind):
    rng = np.random.default_rng(21 + kind)
    for _ in range(20):
        X = rng.standard_normal((4, 3))
        d, g, _ = C.pair_distance(X, kind)
        Q, t = rot(rng), rng.standard_normal(3)
        d2, g2, _ = C.pair_distance(X @ Q.T + t, kind)
        assert d2 == pytest.approx(d, rel=1e-12, abs=1e-14)
        assert np.allclose(g2.reshape(4, 3), g.reshape(4, 3) @ Q.T, atol=1e-9)
        if kind == C.PT:
            d3 = C.pair_distance(X[[0, 2, 3, 1]], kind)[0]
        else:
            d3, g3, _ = C.pair_distance(X[[2, 3, 0, 1]], kind)
            assert np.allclose(g3.reshape(4, 3)[[2, 3, 0, 1]], g.reshape(4, 3), atol=1e-12)
        assert d3 == pytest.approx(d, rel=1e-12, abs=1e-14)


def test_gradient_is_unit_normal_with_weights():
    """|d/dp d| = 1 and the weights of each primitive sum to one (the
    gradient moves the pair rigidly apart at unit rate)."""
    rng = np.random.default_rng(5)
    for kind in (C.PT, C.EE):
        for _ in range(20):
            g = C.pair_distance(rng.standard_normal((4, 3)), kind)[1].reshape(4, 3)
            if kind == C.PT:
                assert np.linalg.norm(g[0]) == pytest.approx(1.0, rel=1e-12)
                assert np.allclose(g.sum(axis=0), 0.0, atol=1e-12)
            else:
                assert np.linalg.norm(g[0] + g[1]) == pytest.approx(1.0, rel=1e-12)
                assert np.allclose(g.sum(axis=0), 0.0, atol=1e-12)
