"""The connectivity-aware hierarchy (supplement Section 1.2) on the device:
the context's vertex order, every level-0 and coarse block, the Woodbury
apply and the PNCG loop against the oracle built on the same order (FP64,
1e-10), on the interleaved combs (two bodies whose Morton runs mix) and
the grid."""
import numpy as np
import pytest

from oracle import fem, mas, woodbury
from paper_2604_19892_amd import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("name,levels", [("combs", 2), ("combs", 3), ("grid", 2)])
def test_blocks_and_apply_match_oracle(name, levels):
    from paper_2604_19892_amd.binding import MasContext, make_config
    print("\n[hierarchy case] %s, %d levels, connectivity order" % (name, levels), flush=True)
    if name == "grid":
        sc = synth.grid_scene()
        base, curr = synth.grid_update_sets(sc)
    else:
        sc = synth.combs_scene()
        d = synth.pool_distance(sc.pool, sc.x)
        base = synth.contact_set(sc.pool['key'], sc.pool['idx'], sc.pool['grad'], d)
        curr = synth.churn_set(np.random.default_rng(5), sc, base, 0.3)
    prob = fem.Problem(sc)
    links = synth.contact_links(sc.pool, sc.x, sc.dhat)
    hier = mas.Hierarchy(sc.X, levels, tets=sc.tets, order="connectivity", links=links)
    H = prob.assemble(sc.x, base)
    M = mas.MAS(hier, H)
    dS, u, _ = woodbury.classify(prob, base, curr)
    sel = woodbury.topk(hier, curr, dS, u, 8)
    blocks = woodbury.updated_blocks(hier, H, curr, u, sel)
    ctx = MasContext(sc, make_config(sc, levels=levels, K=8, hierarchy="connectivity"), links=links)
    try:
        np.testing.assert_array_equal(ctx.perm, hier.perm)
        x = ctx.to_lib(sc.x)
        ctx.build(x, ctx.contacts(base))
        for d in range(hier.num_subdomains(0)):
            Bo = M.fine[d]
            n = Bo.shape[0]
            assert rel(ctx.get_block(0, d)[:n, :n], Bo) < 1e-10, d
        for l in range(1, levels):
            _, _, invs = M.coarse[l - 1]
            for d, (dofs, Minv) in enumerate(invs):
                n = Minv.shape[0]
                assert rel(ctx.get_block(l, d)[:n, :n], Minv) < 1e-10, (l, d)
        ctx.woodbury_update(ctx.contacts(curr))
        g = np.random.default_rng(1).standard_normal(3 * sc.N)
        zo = M.apply(g, blocks)
        zg = ctx.from_lib(ctx.apply(ctx.to_lib(g)))
        assert rel(zg, zo) < 1e-10, rel(zg, zo)
        code, msg = ctx.sync()
        assert code == 0, msg
    finally:
        ctx.close()


def test_loop_matches_oracle_on_the_combs():
    from oracle.solver import OraclePNCG
    from paper_2604_19892_amd.pncg import PNCG
    print("\n[hierarchy case] combs, PNCG loop, connectivity order", flush=True)
    sc = synth.combs_scene()
    ora = OraclePNCG(sc, hierarchy="connectivity")
    gpu = PNCG(sc, block_prec="f64", hierarchy="connectivity")
    for k in range(6):
        ora.iterate()
        gpu.iterate()
        lo, lg = ora.log[-1], gpu.log[-1]
        assert lo["restart"] == lg["restart"], k
        assert lg["mu"] == pytest.approx(lo["mu"], rel=1e-7), k
        assert lg["nu"] == pytest.approx(lo["nu"], rel=1e-6, abs=1e-9), k
        xg = gpu.ctx.from_lib(gpu.x)
        err = np.linalg.norm(xg - ora.x) / np.linalg.norm(ora.x - sc.x.reshape(-1))
        assert err < 1e-6, (k, err)
    code, msg = gpu.ctx.sync()
    assert code == 0, msg
    gpu.ctx.close()
