"""Pins of the brute-force constraint-set oracle (ComputeConstraintSet of
Algorithm 1): the box-distance prune is a lower bound, the pruned search
equals the unpruned one on a small two-box mesh, hand-built cases."""
import numpy as np
import pytest

from oracle import constraint_set as CS
from oracle import contact as C
from paper_2604_19892_amd import synth


def test_box_distance_is_a_lower_bound():
    rng = np.random.default_rng(1)
    for kind in (C.PT, C.EE):
        for _ in range(200):
            X = rng.standard_normal((4, 3))
            A, B = (X[:1], X[1:]) if kind == C.PT else (X[:2], X[2:])
            bd = CS.box_distance(A.min(0), A.max(0), B.min(0), B.max(0))
            assert bd <= C.pair_distance(X, kind)[0] + 1e-15
    assert CS.box_distance(np.zeros(3), np.ones(3), 0.5 * np.ones(3), 2 * np.ones(3)) == 0.0
    assert CS.box_distance(np.zeros(3), np.ones(3), np.array([4.0, 1.0, 1.0]), 5 * np.ones(3)) == 3.0


def unpruned(x, verts, tris, edges, dhat):
    X = x.reshape(-1, 3)
    rows = []
    for v in verts:
        for t in tris:
            if v in t:
                continue
            ids = np.array([v, *t])
            d = C.pair_distance(X[ids], C.PT)[0]
            if d < dhat:
                rows.append((0, *ids))
    for a in range(len(edges)):
        for b in range(a + 1, len(edges)):
            if len({*edges[a], *edges[b]}) < 4:
                continue
            ids = np.array([*edges[a], *edges[b]])
            d = C.pair_distance(X[ids], C.EE)[0]
            if d < dhat:
                rows.append((1, *ids))
    return sorted(rows)


def test_pruned_equals_unpruned_on_small_boxes():
    sc = synth.two_boxes_scene(nxy=4, nz=3, n_contacts=20)
    verts, tris, edges = synth.surface(sc.tets)
    dhat = sc.dhat
    pairs, kinds, d = CS.constraint_set(sc.x, verts, tris, edges, dhat)
    got = sorted((int(k), *map(int, p)) for k, p in zip(kinds, pairs))
    want = unpruned(sc.x, verts, tris, edges, dhat)
    assert got == want
    assert len(want) > 10 and {r[0] for r in want} == {0, 1}
    assert np.all(d < dhat)


def test_hand_built_cases():
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.2, 0.2, 0.0], [0.5, -0.5, 0], [0.5, 0.5, 0]], float)
    tris = np.array([[0, 1, 2]])
    edges = np.array([[0, 1], [4, 5]])
    verts = np.array([0, 1, 2, 3, 4, 5])
    for h in (5e-4, 2e-3):
        Y = X.copy()
        Y[3, 2] = h        # point above the face
        Y[4:, 2] = -h      # an edge crossing below edge 0-1; vertex 5 lies under the hypotenuse
        pairs, kinds, d = CS.constraint_set(Y, verts, tris, edges, 1e-3)
        assert int((kinds == C.PT).sum()) == (2 if h < 1e-3 else 0)
        if h < 1e-3:
            assert [3, 0, 1, 2] in pairs.tolist() and [5, 0, 1, 2] in pairs.tolist()
            assert [0, 1, 4, 5] in pairs.tolist()
            assert d[kinds == C.EE][0] == pytest.approx(h, abs=1e-15)
        else:
            assert pairs.shape[0] == 0
    # pairs that share a vertex are never contacts
    pairs, kinds, _ = CS.constraint_set(X, verts, tris, np.array([[0, 1], [1, 2]]), 1e-3)
    for p, k in zip(pairs, kinds):
        if k == C.PT:
            assert p[0] not in p[1:]
        else:
            assert len(set(p.tolist())) == 4
