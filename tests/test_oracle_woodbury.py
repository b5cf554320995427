"""Pins of the oracle's classification, Top-K and updated fine blocks.

Anchors: one hand-built contact per classification branch, a brute-force
ranking written independently of the oracle's, the Sherman-Morrison closed
form for a single update vector, and the Woodbury formula (evaluated here
from a separately inverted base block) against the oracle's direct
inversion of the updated block.
"""
import itertools

import numpy as np
import pytest

from oracle import fem, mas, woodbury
from paper_2604_19892_amd import synth


def _one(key, v, n, d):
    idx = np.array([[v, -1, -1, -1]], np.int32)
    g = np.zeros((1, 12))
    g[0, :3] = n
    return synth.contact_set(np.array([key], np.uint64), idx, g, np.array([d]))


def test_classification_branches(grid):
    prob = fem.Problem(grid)
    n = np.array([0.0, 0.0, 1.0])
    base = synth.concat(_one(1, 10, n, 5e-4), _one(2, 11, n, 5e-4), _one(3, 12, n, 5e-4),
                        _one(4, 13, n, 5e-4))
    th = np.deg2rad(40.0)
    n_rot = np.array([np.sin(th), 0.0, np.cos(th)])
    th2 = np.deg2rad(20.0)
    n_small = np.array([np.sin(th2), 0.0, np.cos(th2)])
    curr = synth.concat(
        _one(1, 10, n, 2.5e-4),        # stiffening (closer)
        _one(2, 11, n, 8e-4),          # softening (farther)
        _one(3, 12, n_rot, 5e-4),      # rotated by 40 degrees > 25
        _one(4, 13, n_small, 1e-4),    # rotated by 20 degrees < 25, stiffer
        _one(9, 20, n, 3e-4),          # new
        _one(10, 21, n, 2e-3),         # new but beyond dhat: k = 0
    )
    dS, u, case = woodbury.classify(prob, base, curr)
    k = lambda d: prob.kappa * fem.barrier(np.array([d]), prob.dhat)[2][0]
    assert list(case[:5]) == [woodbury.STIFFEN, woodbury.SOFTEN, woodbury.ROTATED,
                              woodbury.STIFFEN, woodbury.NEW]
    assert dS[0] == pytest.approx(k(2.5e-4) - k(5e-4), rel=1e-13)
    assert dS[1] == 0 and np.all(u[1] == 0)
    assert dS[2] == pytest.approx(k(5e-4), rel=1e-13)
    np.testing.assert_allclose(u[2, :3], np.sqrt(k(5e-4)) * n_rot, rtol=1e-13)
    assert dS[3] == pytest.approx(k(1e-4) - k(5e-4), rel=1e-13)
    assert dS[4] == pytest.approx(k(3e-4), rel=1e-13)
    assert dS[5] == 0                  # released / inactive contact adds nothing
    # u u^T carries exactly the stiffness increment along n
    assert float(u[0] @ u[0]) == pytest.approx(dS[0], rel=1e-13)


def test_topk_matches_brute_force(grid):
    prob = fem.Problem(grid)
    hier = mas.Hierarchy(grid.X, 2)
    rng = np.random.default_rng(11)
    # many contacts crowded onto few vertices so that subdomains overflow K
    m = 400
    idx = np.full((m, 4), -1, np.int32)
    idx[:, 0] = rng.integers(0, 64, m)
    idx[:, 1] = rng.integers(0, 512, m)
    grad = rng.standard_normal((m, 12))
    grad[:, 6:] = 0
    d = rng.uniform(1e-5, 1e-3, m)
    d[::7] = d[3]                          # ties in dS broken by key
    keys = rng.permutation(10 ** 6)[:m].astype(np.uint64)
    curr = synth.contact_set(keys, idx, grad, d)
    base = synth.contact_set(np.zeros(0, np.uint64), np.zeros((0, 4), np.int32), np.zeros((0, 12)), np.zeros(0))
    dS, u, _ = woodbury.classify(prob, base, curr)
    K = 8
    sel = woodbury.topk(hier, curr, dS, u, K)
    # brute force: all (subdomain, contact) incidences, full sort per subdomain
    inc = {}
    for c in range(m):
        for v in set(int(q) for q in idx[c] if q >= 0):
            inc.setdefault(int(hier.rank[v] // 32), set()).add(c)
    assert set(sel) == set(inc)
    for dd, cs in inc.items():
        order = sorted(cs, key=lambda c: (-dS[c], int(keys[c])))
        assert sel[dd] == order[:K]
        assert len(sel[dd]) == min(K, len(cs))


def test_sherman_morrison_single_vector(grid):
    prob = fem.Problem(grid)
    hier = mas.Hierarchy(grid.X, 2)
    base, _ = synth.grid_update_sets(grid)
    H = prob.assemble(grid.x, base)
    # one new contact on a vertex of subdomain 3
    v = int(hier.perm[3 * 32 + 5])
    curr = _one(777, v, np.array([0.6, 0.0, 0.8]), 2e-5)
    dS, u, _ = woodbury.classify(prob, base, curr)
    sel = woodbury.topk(hier, curr, dS, u, 8)
    assert sel == {3: [0]}
    blocks = woodbury.updated_blocks(hier, H, curr, u, sel)
    dofs = hier.subdomain_dofs(3)
    B = np.linalg.inv(H[dofs][:, dofs].toarray())
    ud = np.zeros(dofs.size)
    ud[15:18] = u[0, :3]
    Bu = B @ ud
    sm = B - np.outer(Bu, Bu) / (1.0 + ud @ Bu)
    np.testing.assert_allclose(blocks[3], sm, rtol=1e-9, atol=1e-12 * np.abs(sm).max())
    # untouched subdomains keep their base inverse
    d0 = hier.subdomain_dofs(0)
    np.testing.assert_allclose(blocks[0], np.linalg.inv(H[d0][:, d0].toarray()), rtol=1e-12)


def test_woodbury_formula_equals_direct_inverse(grid):
    prob = fem.Problem(grid)
    hier = mas.Hierarchy(grid.X, 2)
    base, curr = synth.grid_update_sets(grid)
    H = prob.assemble(grid.x, base)
    dS, u, case = woodbury.classify(prob, base, curr)
    # every branch of the classification occurs in the scripted update
    assert {woodbury.NEW, woodbury.ROTATED, woodbury.STIFFEN, woodbury.SOFTEN} <= set(case.tolist())
    sel = woodbury.topk(hier, curr, dS, u, 8)
    blocks = woodbury.updated_blocks(hier, H, curr, u, sel)
    for d, cols in sel.items():
        dofs = hier.subdomain_dofs(d)
        B = np.linalg.inv(H[dofs][:, dofs].toarray())
        Ud = woodbury.local_U(hier, curr, u, d, cols)
        W = B @ Ud
        Cap = np.eye(len(cols)) + Ud.T @ W
        Bt = B - W @ np.linalg.solve(Cap, W.T)
        np.testing.assert_allclose(blocks[d], Bt, rtol=1e-8, atol=1e-10 * np.abs(Bt).max())
