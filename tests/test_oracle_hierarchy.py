"""Pins of the connectivity-aware hierarchy order (supplement Section 1.2,
the reading in oracle/mas.py): hand-worked aggregations, runs on a path,
the partial last node, interleaved chains that Morton runs mix and the
connectivity order keeps apart, and the structural invariants of the order
(a permutation; level-l nodes are runs of 32^l vertices; at most one
level-0 subdomain per component boundary mixes components)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from oracle import mas


def _adj(n, edges):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    return adj


def test_hand_aggregations():
    # seed 0 takes 1 (smallest neighbour), then 2; seed 3 takes 4 then 5
    adj = _adj(6, [(0, 1), (0, 2), (1, 2), (2, 3), (3, 4), (4, 5), (1, 5)])
    assert mas.aggregate(adj, 6, 3) == [[0, 1, 2], [3, 4, 5]]
    # seed 0: {3, 5} -> 3, {4, 5} -> 4; seed 1: {5} -> 5, then no unassigned
    # neighbour: the smallest unassigned node, 2
    adj = _adj(6, [(0, 5), (0, 3), (5, 1), (3, 4)])
    assert mas.aggregate(adj, 6, 3) == [[0, 3, 4], [1, 5, 2]]


def test_path_and_partial_last_node():
    adj = _adj(70, [(i, i + 1) for i in range(69)])
    cl = mas.aggregate(adj, 70)
    assert cl == [list(range(0, 32)), list(range(32, 64)), list(range(64, 70))]
    # the partial node joins the last cluster at its end
    cl = mas.aggregate(adj, 70, partial_last=True)
    assert cl[-1] == list(range(64, 70)) and [len(c) for c in cl] == [32, 32, 6]
    # ... or starts its own when that cluster is full
    adj = _adj(65, [(i, i + 1) for i in range(64)])
    cl = mas.aggregate(adj, 65, partial_last=True)
    assert [len(c) for c in cl] == [32, 32, 1] and cl[-1] == [64]


def _interleaved_chains(n):
    """Vertices on a line (Morton rank = position); even positions form one
    chain, odd positions another (degenerate tets carry the edges)."""
    X = np.zeros((n, 3))
    X[:, 0] = np.arange(n)
    tets = np.array([[r, r + 2, r + 2, r + 2] for r in range(n - 2)], np.int64)
    return X, tets


def test_interleaved_chains_are_not_mixed():
    X, tets = _interleaved_chains(128)
    perm = mas.connectivity_perm(X, tets, 1)
    runs = (perm % 2).reshape(-1, 32)
    assert np.all(runs == runs[:, :1])                 # one chain per subdomain
    np.testing.assert_array_equal(perm[:32], np.arange(0, 64, 2))
    mort = (mas.morton_perm(X) % 2).reshape(-1, 32)
    assert np.all(mort.min(1) != mort.max(1))           # Morton runs mix both


def test_contact_links_join_the_graph():
    # links between every pair of neighbouring positions make the two
    # chains one path: the clusters are runs of consecutive positions
    X, tets = _interleaved_chains(128)
    links = np.array([[r, r + 1] for r in range(127)])
    perm = mas.connectivity_perm(X, tets, 1, links=links)
    np.testing.assert_array_equal(perm, np.arange(128))
    # a single link merges the components: component-major numbering then
    # keeps the chain of the smallest rank first only up to the link
    perm1 = mas.connectivity_perm(X, tets, 1, links=np.array([[0, 1]]))
    assert perm1[0] == 0 and perm1[1] == 1


def _components(X, tets):
    t = np.asarray(tets, np.int64)
    rows = np.repeat(t, 4, axis=1).ravel()
    cols = np.tile(t, (1, 4)).ravel()
    A = sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(X.shape[0],) * 2).tocsr()
    return connected_components(A, directed=False)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_structure_on_the_combs(levels):
    from paper_2604_19892_amd import synth
    sc = synth.combs_scene()
    perm = mas.connectivity_perm(sc.X, sc.tets, levels)
    np.testing.assert_array_equal(np.sort(perm), np.arange(sc.N))
    ncomp, lab = _components(sc.X, sc.tets)
    assert ncomp == 2
    runs = lab[perm[:(sc.N // 32) * 32]].reshape(-1, 32)
    mixed = int((runs.min(1) != runs.max(1)).sum())
    assert mixed <= ncomp - 1
    # level-l nodes: the clusters of level l-1, 32^l vertices each but the last
    mperm, cls = mas.connectivity_clusters(sc.X, sc.tets, levels)
    sizes = np.ones(sc.N, np.int64)
    for l, cl in enumerate(cls):
        assert sorted(m for c in cl for m in c) == list(range(len(sizes)))
        sizes = np.array([sizes[c].sum() for c in cl])
        assert np.all(sizes[:-1] == 32 ** (l + 1)) and 0 < sizes[-1] <= 32 ** (l + 1)
    # Morton runs on the same scene mix the combs in most subdomains
    mort = lab[mas.morton_perm(sc.X)[:(sc.N // 32) * 32]].reshape(-1, 32)
    assert int((mort.min(1) != mort.max(1)).sum()) > runs.shape[0] // 2


def test_hierarchy_uses_the_order():
    from paper_2604_19892_amd import synth
    sc = synth.grid_scene()
    h = mas.Hierarchy(sc.X, 2, tets=sc.tets, order="connectivity")
    np.testing.assert_array_equal(h.perm, mas.connectivity_perm(sc.X, sc.tets, 2))
    assert h.subdomain_of_vertex(h.perm[33]) == 1
    with pytest.raises(ValueError):
        mas.Hierarchy(sc.X, 2, order="other")
