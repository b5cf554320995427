"""GPU parity of ComputeConstraintSet (Algorithm 1; broad phase by hashed
grid, narrow phase by closest features) against the brute-force oracle.

Small meshes: the set of pairs found is identical (pairs whose distance is
within 1e-12 of dhat may fall either way and are left out of the
comparison).  The full two-box mesh: every pair found is a contact, none
twice, none sharing a vertex, and for sampled surface vertices and edges
the pairs found are exactly the brute-force ones."""
import numpy as np
import pytest

from oracle import constraint_set as CS
from oracle import contact as C
from paper_2604_19892_amd import synth

pytestmark = pytest.mark.gpu


def gpu_set(ctx, x, verts, tris, edges, dhat, cap=None):
    import torch
    dev = "cuda"
    r = ctx.rank
    vt = torch.as_tensor(r[verts].astype(np.int32), device=dev)
    tt = torch.as_tensor(r[tris].astype(np.int32).reshape(-1, 3), device=dev)
    et = torch.as_tensor(r[edges].astype(np.int32).reshape(-1, 2), device=dev)
    cap = cap if cap is not None else 4 * (len(verts) + len(edges)) + 1024
    pairs = torch.full((cap, 4), -1, dtype=torch.int32, device=dev)
    kind = torch.zeros(cap, dtype=torch.uint8, device=dev)
    dist = torch.zeros(cap, dtype=torch.float64, device=dev)
    grad = torch.zeros(cap, 12, dtype=torch.float64, device=dev)
    key = torch.zeros(cap, dtype=torch.int64, device=dev)
    n = ctx.constraint_set(ctx.to_lib(x), vt, tt, et, dhat, pairs, kind, dist, grad, key)
    code, msg = ctx.sync()
    assert code == 0, msg
    k = min(n, cap)
    inv = np.argsort(r)  # library id -> original id
    P = inv[pairs[:k].cpu().numpy()]
    check_keys(key[:k].cpu().numpy().view(np.uint64), P, kind[:k].cpu().numpy(), verts, tris, edges)
    return n, P, kind[:k].cpu().numpy(), dist[:k].cpu().numpy(), grad[:k].cpu().numpy()


def check_keys(keys, P, K, verts, tris, edges):
    """Each pair's key names its two primitives in the lists given: tag 2
    point-triangle (vertex index, triangle index), tag 3 edge-edge (the
    two edge indices, smaller first); no key twice."""
    assert len(np.unique(keys)) == len(keys)
    tag = keys >> np.uint64(60)
    a = ((keys >> np.uint64(30)) & np.uint64((1 << 30) - 1)).astype(np.int64)
    b = (keys & np.uint64((1 << 30) - 1)).astype(np.int64)
    tris = np.asarray(tris).reshape(-1, 3)
    edges = np.asarray(edges).reshape(-1, 2)
    for t, i, j, p, k in zip(tag, a, b, P, K):
        assert int(t) == 2 + int(k)
        if k == C.PT:
            assert verts[i] == p[0] and list(tris[j]) == list(p[1:])
        else:
            assert i < j and list(edges[i]) == list(p[:2]) and list(edges[j]) == list(p[2:])


def as_rows(P, K):
    return [(int(k), *map(int, p)) for p, k in zip(P, K)]


def edge_pair_key(p, k):
    """Edge-edge pairs as reported: edges as given, first edge by its index;
    normalised here to the sorted vertex pairs, so both sides compare."""
    if k == C.PT:
        return (0, p[0], *sorted(p[1:]))
    a, b = tuple(sorted(p[:2])), tuple(sorted(p[2:]))
    return (1, *min(a, b), *max(a, b))


def check_found(X, P, K, d, g, dhat):
    """Every pair found is a contact with the oracle's distance; no
    duplicates; no shared vertex."""
    keys = [edge_pair_key(p, k) for p, k in zip(P, K)]
    assert len(set(keys)) == len(keys)
    for p, k, dd in zip(P, K, d):
        assert len(set(p.tolist())) == 4
        do = C.pair_distance(X[p], k)[0]
        ext = np.linalg.norm(X[p].max(0) - X[p].min(0))
        assert abs(dd - do) <= 1e-12 * ext
        assert do < dhat + 1e-12 * ext
    return set(keys)


def test_small_two_boxes_exact_set():
    from paper_2604_19892_amd.binding import MasContext, make_config
    sc = synth.two_boxes_scene(nxy=10, nz=5, n_contacts=200)
    verts, tris, edges = synth.surface(sc.tets)
    edge = 1.0 / 9
    ctx = MasContext(sc, make_config(sc, levels=2, K=8))
    try:
        for dhat in (sc.dhat, 0.3 * edge):
            print("\n[constraint set case] two boxes 10x10x5, dhat %.3g" % dhat, flush=True)
            n, P, K, d, g = gpu_set(ctx, sc.x, verts, tris, edges, dhat)
            X = sc.x.reshape(-1, 3)
            got = check_found(X, P, K, d, g, dhat)
            po, ko, do = CS.constraint_set(sc.x, verts, tris, edges, dhat)
            want = {edge_pair_key(p, k) for p, k in zip(po, ko)}
            # pairs at dhat within rounding may go either way
            border = set()
            for key in got ^ want:
                k = key[0]
                ids = np.array(key[1:])
                assert abs(C.pair_distance(X[ids], k)[0] - dhat) <= 1e-12, key
                border.add(key)
            print("pairs %d (PT %d, EE %d), border %d" % (n, int((K == 0).sum()), int((K == 1).sum()), len(border)))
            assert n == len(P) and len(want) > 50 and {0, 1} <= set(ko.tolist())
    finally:
        ctx.close()


def test_full_two_boxes_sampled():
    from paper_2604_19892_amd.binding import MasContext, make_config
    sc = synth.two_boxes_scene()
    verts, tris, edges = synth.surface(sc.tets)
    dhat = sc.dhat
    print("\n[constraint set case] two boxes 40x40x20, %d verts %d tris %d edges" % (
        len(verts), len(tris), len(edges)), flush=True)
    ctx = MasContext(sc, make_config(sc, levels=2, K=8))
    try:
        n, P, K, d, g = gpu_set(ctx, sc.x, verts, tris, edges, dhat)
        X = sc.x.reshape(-1, 3)
        rng = np.random.default_rng(4)
        sample = rng.choice(n, min(n, 3000), replace=False)
        check_found(X, P[sample], K[sample], d[sample], g[sample], dhat)
        keys = [edge_pair_key(p, k) for p, k in zip(P, K)]
        assert len(set(keys)) == len(keys)
        print("pairs %d (PT %d, EE %d)" % (n, int((K == 0).sum()), int((K == 1).sum())))
        assert (K == 0).sum() > 1000 and (K == 1).sum() > 1000
        # completeness for sampled vertices and edges against brute force
        sv = rng.choice(verts, 150, replace=False)
        po, ko, _ = CS.constraint_set(sc.x, sv, tris, np.zeros((0, 2), np.int64), dhat)
        want = {edge_pair_key(p, k) for p, k in zip(po, ko)}
        got = {kk for kk in keys if kk[0] == 0 and kk[1] in set(sv.tolist())}
        for key in got ^ want:
            assert abs(C.pair_distance(X[np.array(key[1:])], C.PT)[0] - dhat) <= 1e-12, key
        assert len(want) > 20
        se = edges[rng.choice(len(edges), 150, replace=False)]
        E = X[edges]
        lo, hi = E.min(1), E.max(1)
        want = set()
        for e in se:
            bd = CS.box_distance(X[e].min(0), X[e].max(0), lo, hi)
            for j in np.nonzero(bd < dhat)[0]:
                f = edges[j]
                if len({*e, *f}) < 4:
                    continue
                ids = np.array([*e, *f])
                if C.pair_distance(X[ids], C.EE)[0] < dhat:
                    want.add(edge_pair_key(ids, C.EE))
        sset = {tuple(sorted(e)) for e in se}
        got = {kk for kk in keys if kk[0] == 1 and (tuple(kk[1:3]) in sset or tuple(kk[3:5]) in sset)}
        for key in got ^ want:
            assert abs(C.pair_distance(X[np.array(key[1:])], C.EE)[0] - dhat) <= 1e-12, key
        assert len(want) > 20
    finally:
        ctx.close()


def test_capacity_empty_and_errors():
    import torch
    from paper_2604_19892_amd.binding import MasContext, make_config
    from paper_2604_19892_amd._abi import MasError
    sc = synth.two_boxes_scene(nxy=10, nz=5, n_contacts=200)
    verts, tris, edges = synth.surface(sc.tets)
    ctx = MasContext(sc, make_config(sc, levels=2, K=8))
    try:
        print("\n[constraint set case] capacity 10, empty surface, bad id, NaN", flush=True)
        dhat = 0.3 / 9
        n_all, P_all, K_all, _, _ = gpu_set(ctx, sc.x, verts, tris, edges, dhat)
        n, P, K, d, _ = gpu_set(ctx, sc.x, verts, tris, edges, dhat, cap=10)
        assert n == n_all and len(P) == 10
        all_keys = {edge_pair_key(p, k) for p, k in zip(P_all, K_all)}
        assert {edge_pair_key(p, k) for p, k in zip(P, K)} <= all_keys
        e0 = np.zeros(0, np.int64)
        n0, _, _, _, _ = gpu_set(ctx, sc.x, verts, e0.reshape(0, 3), e0.reshape(0, 2), dhat)
        assert n0 == 0
        dev = "cuda"
        x = ctx.to_lib(sc.x)
        vt = torch.as_tensor(np.array([0, 1, sc.N], np.int32), device=dev)
        tt = torch.as_tensor(np.array([[2, 3, 4]], np.int32), device=dev)
        et = torch.zeros(0, 2, dtype=torch.int32, device=dev)
        pairs = torch.zeros(4, 4, dtype=torch.int32, device=dev)
        kind = torch.zeros(4, dtype=torch.uint8, device=dev)
        dist = torch.zeros(4, dtype=torch.float64, device=dev)
        with pytest.raises(MasError):
            ctx.constraint_set(x, vt, tt, et, dhat, pairs, kind, dist)
        xn = x.clone()
        xn[3 * 3] = float("nan")
        with pytest.raises(MasError):
            ctx.constraint_set(xn, vt[:2], tt, et, dhat, pairs, kind, dist)
        assert ctx.sync()[0] == 0
    finally:
        ctx.close()
