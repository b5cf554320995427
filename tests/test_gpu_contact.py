"""GPU parity of the contact narrow phase (distance d_c, n = grad d_c and
closest-feature type of point-triangle and edge-edge pairs; Sections 3.1
and 4.1) against the FP64 oracle.

The oracle tries every candidate sub-simplex and keeps the nearest; the
kernel locates the closest point by Voronoi regions.  Distances agree to
rounding (1e-12 of the pair's extent).  Gradients are unique wherever the
closest points are (point-triangle pairs with d > 0 and a triangle with
area, edge-edge pairs that are not parallel) and agree to 1e-9 of
extent / d there.  Types are compared where the oracle's type does not change under perturbations of
1e-9 of the extent (elsewhere either feature is correct)."""
import numpy as np
import pytest

from oracle import contact as C
from paper_2604_19892_amd import synth

pytestmark = pytest.mark.gpu


def pool_pairs(sc):
    idx = sc.pool["idx"].astype(np.int64)
    tag = (sc.pool["key"] >> np.uint64(60)).astype(np.int64)
    keep = (tag == synth.KEY_PT) | (tag == synth.KEY_EE)
    kinds = np.where(tag[keep] == synth.KEY_PT, C.PT, C.EE).astype(np.uint8)
    return idx[keep], kinds


def run_gpu(ctx, x, pairs, kinds):
    import torch
    dev = "cuda"
    m = pairs.shape[0]
    lib_pairs = torch.as_tensor(ctx.rank[pairs].astype(np.int32).reshape(m, 4), device=dev)
    kind_t = torch.as_tensor(kinds, device=dev)
    dist = torch.zeros(m, dtype=torch.float64, device=dev)
    grad = torch.zeros(m, 12, dtype=torch.float64, device=dev)
    ty = torch.zeros(m, dtype=torch.uint8, device=dev)
    ctx.contact_distances(ctx.to_lib(x), lib_pairs, kind_t, dist, grad, ty)
    code, msg = ctx.sync()
    return code, msg, dist.cpu().numpy(), grad.cpu().numpy(), ty.cpu().numpy().astype(np.int64)


def compare(X, pairs, kinds, d, g, ty, type_sample=3000):
    do, go, to = C.contact_distances(X, pairs, kinds)
    P = X[pairs]  # (m, 4, 3)
    ext = np.linalg.norm(P.max(axis=1) - P.min(axis=1), axis=1)
    assert np.all(np.abs(d - do) <= 1e-12 * ext + 1e-300), np.max(np.abs(d - do) / ext)
    u = P[:, 1] - P[:, 0]
    v = P[:, 3] - P[:, 2]
    sin2 = np.sum(np.cross(u, v) ** 2, axis=1) / np.maximum(np.sum(u * u, 1) * np.sum(v * v, 1), 1e-300)
    e1, e2 = P[:, 2] - P[:, 1], P[:, 3] - P[:, 1]
    tri = np.sum(np.cross(e1, e2) ** 2, axis=1) / np.maximum(np.sum(e1 * e1, 1) * np.sum(e2 * e2, 1), 1e-300)
    # closest points unique: a triangle with area (else its barycentric
    # weights are not), edges that are not parallel
    unique = (do > 1e-9 * ext) & np.where(kinds == C.PT, tri > 1e-6, sin2 > 1e-6)
    tol = 1e-9 * ext / np.maximum(do, 1e-300)
    gerr = np.max(np.abs(g - go), axis=1)
    bad = np.nonzero(unique & (gerr > tol))[0]
    assert bad.size == 0, (bad[:5], gerr[bad[:5]], tol[bad[:5]], kinds[bad[:5]], ty[bad[:5]], to[bad[:5]])
    # types where the oracle's is stable under small perturbations
    rng = np.random.default_rng(3)
    sample = rng.choice(pairs.shape[0], min(type_sample, pairs.shape[0]), replace=False)
    stable = 0
    for i in sample:
        x4 = X[pairs[i]]
        if all(C.pair_distance(x4 + 1e-9 * ext[i] * rng.standard_normal((4, 3)), kinds[i])[2] == to[i]
               for _ in range(3)):
            stable += 1
            assert ty[i] == to[i], (i, ty[i], to[i])
    return unique.mean(), stable / len(sample), np.max(np.abs(d - do) / ext)


def test_two_box_scene_pairs():
    from paper_2604_19892_amd.binding import MasContext, make_config
    sc = synth.two_boxes_scene()
    pairs, kinds = pool_pairs(sc)
    print("\n[contact case] two boxes, %d pairs" % pairs.shape[0], flush=True)
    ctx = MasContext(sc, make_config(sc, levels=2, K=8))
    try:
        code, msg, d, g, ty = run_gpu(ctx, sc.x, pairs, kinds)
        assert code == 0, msg
        X = sc.x.reshape(-1, 3)
        fu, fs, derr = compare(X, pairs, kinds, d, g, ty)
        print("unique gradients %.3f, stable types %.3f, max rel d err %.2e" % (fu, fs, derr))
        assert fu > 0.9 and fs > 0.9
        # every feature type occurs on this scene's pairs or the random ones below
        assert len(np.unique(ty)) >= 4
    finally:
        ctx.close()


def test_random_pairs_and_degenerate_cases():
    from paper_2604_19892_amd.binding import MasContext, make_config
    sc = synth.two_boxes_scene()
    ctx = MasContext(sc, make_config(sc, levels=2, K=8))
    try:
        rng = np.random.default_rng(17)
        N = sc.N
        X = rng.uniform(-1.0, 1.0, (N, 3))
        # hand-placed degenerate primitives on vertices 0..15
        X[0:4] = [[0.25, 0.25, 0.0], [0, 0, 0], [1, 0, 0], [0, 1, 0]]           # point on the face: d = 0
        X[4:8] = [[1.5, 0.7, 0.0], [0, 0, 0], [1, 0, 0], [2, 0, 0]]             # collinear triangle
        X[8:12] = [[0, 0, 0], [1, 0, 0], [0.5, 1, 0], [1.5, 1, 0]]              # parallel edges
        X[12:16] = [[0.3, 2, 0], [0.3, 2, 0], [0, 0, 0], [1, 0, 0]]             # zero-length edge
        special = np.array([[0, 1, 2, 3], [4, 5, 6, 7], [8, 9, 10, 11], [12, 13, 14, 15]])
        skind = np.array([C.PT, C.PT, C.EE, C.EE], np.uint8)
        m = 5003  # ragged: not a multiple of the 256-thread workgroup
        rp = np.stack([rng.choice(np.arange(16, N), 4, replace=False) for _ in range(m)])
        rk = rng.integers(0, 2, m).astype(np.uint8)
        pairs = np.concatenate([special, rp])
        kinds = np.concatenate([skind, rk])
        print("\n[contact case] random cloud, %d pairs incl. 4 degenerate" % pairs.shape[0], flush=True)
        code, msg, d, g, ty = run_gpu(ctx, X.reshape(-1), pairs, kinds)
        assert code == 0, msg
        assert d[0] == 0.0 and not g[0].any()
        assert d[1] == pytest.approx(0.7, abs=1e-15)
        assert d[2] == pytest.approx(1.0, abs=1e-15)
        assert d[3] == pytest.approx(2.0, abs=1e-15)
        fu, fs, derr = compare(X, pairs, kinds, d, g, ty, type_sample=2000)
        print("unique gradients %.3f, stable types %.3f, max rel d err %.2e" % (fu, fs, derr))
        assert len(np.unique(ty[4:][kinds[4:] == C.PT])) == 7
        assert len(np.unique(ty[4:][kinds[4:] == C.EE])) >= 5
    finally:
        ctx.close()


def test_empty_call_and_out_of_range_ids():
    import torch
    from paper_2604_19892_amd.binding import MasContext, make_config
    sc = synth.two_boxes_scene()
    ctx = MasContext(sc, make_config(sc, levels=2, K=8))
    try:
        print("\n[contact case] empty call, then one pair naming vertex N", flush=True)
        dev = "cuda"
        x = ctx.to_lib(sc.x)
        empty_i = torch.zeros(0, 4, dtype=torch.int32, device=dev)
        empty_k = torch.zeros(0, dtype=torch.uint8, device=dev)
        empty_d = torch.zeros(0, dtype=torch.float64, device=dev)
        ctx.contact_distances(x, empty_i, empty_k, empty_d)
        assert ctx.sync()[0] == 0
        bad = torch.tensor([[0, 1, 2, sc.N]], dtype=torch.int32, device=dev)
        kind = torch.zeros(1, dtype=torch.uint8, device=dev)
        dist = torch.zeros(1, dtype=torch.float64, device=dev)
        ty = torch.zeros(1, dtype=torch.uint8, device=dev)
        ctx.contact_distances(x, bad, kind, dist, None, ty)
        code, msg = ctx.sync()
        assert code == 1, msg  # MAS_ERR_INVALID_ARG
        assert np.isnan(dist.cpu().numpy()[0]) and int(ty.cpu().numpy()[0]) == 255
        # the CCD of the same pair: step 0, reported the same way
        p = torch.zeros_like(x)
        ap = torch.ones(1, dtype=torch.float64, device=dev)
        ctx.ccd_steps(x, p, bad, kind, dist, ap)
        code, msg = ctx.sync()
        assert code == 1, msg
        assert ap.cpu().numpy()[0] == 0.0
        assert ctx.sync()[0] == 0  # the flag was cleared
    finally:
        ctx.close()
