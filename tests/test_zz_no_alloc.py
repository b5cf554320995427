"""pncg_subspace_step_noalloc: the subspace step with the library's fixed
device workspace gives the same results as pncg_subspace_step, bit for bit,
on two calls in a row (a 64,000-vertex scene, then a 512-vertex one, so the
second call finds the first call's larger contents in the shared array), in
the restart form and the two-direction form with an update in H~.
"""
import numpy as np
import pytest

from paper_2604_19892_amd import synth

pytestmark = pytest.mark.gpu


def scene_sets(name):
    if name == "grid":
        sc = synth.grid_scene()
        base, curr = synth.grid_update_sets(sc)
        return sc, base, curr, 2
    sc = synth.two_boxes_scene()
    rng = np.random.default_rng(5)
    d = synth.pool_distance(sc.pool, sc.x)
    base = synth.contact_set(sc.pool['key'], sc.pool['idx'], sc.pool['grad'], d)
    curr = synth.churn_set(rng, sc, base, 0.3)
    return sc, base, curr, 3


def compare_steps(name):
    import torch
    from paper_2604_19892_amd.binding import MasContext, make_config
    print("\n[no-alloc case] %s" % name, flush=True)
    sc, base, curr, L = scene_sets(name)
    ctx = MasContext(sc, make_config(sc, levels=L, K=8))
    x = ctx.to_lib(sc.x)
    ctx.build(x, ctx.contacts(base))
    ctx.woodbury_update(ctx.contacts(curr))
    rng = np.random.default_rng(11)
    g = ctx.to_lib(rng.standard_normal(3 * sc.N))
    zp = ctx.to_lib(rng.standard_normal(3 * sc.N))
    # the second step takes a new z, so that p (a multiple of the first z)
    # and z span a plane
    zs = [ctx.apply(g), ctx.apply(ctx.to_lib(rng.standard_normal(3 * sc.N)))]
    vzs = [ctx.hess_vec(z, with_update=False) for z in zs]
    out_a = torch.zeros_like(ctx.out)
    out_b = torch.zeros_like(ctx.out)
    pa, vpa = ctx.vec(), ctx.vec()
    pb, vpb = ctx.vec(), ctx.vec()
    for restart, zprev, z, vz in ((1, None, zs[0], vzs[0]), (0, zp, zs[1], vzs[1])):
        # the fixed-workspace call first, then the context's own
        ctx.subspace_step_noalloc(g, z, zprev, vz, pb, vpb, restart, out_b)
        ctx.subspace_step(g, z, zprev, vz, pa, vpa, restart)
        out_a.copy_(ctx.out)
        code, msg = ctx.sync()
        assert code == 0, msg
        sa, sb = ctx.step_out(out_a), ctx.step_out(out_b)
        assert np.isfinite(sa["mu"]) and sa["mu"] != 0.0
        assert sa == sb, (restart, sa, sb)
        assert torch.equal(pa, pb) and torch.equal(vpa, vpb), restart
        if not restart:
            assert sa["nu"] != 0.0 and sa["restart_used"] == 0 and sa["fallback"] == 0
    ctx.close()


def test_noalloc_step_matches_step_on_two_calls_in_a_row():
    compare_steps("boxes")
    compare_steps("grid")


def test_noalloc_step_needs_a_build():
    import torch
    from paper_2604_19892_amd import _abi
    from paper_2604_19892_amd.binding import MasContext, make_config, _ptr
    sc = synth.grid_scene()
    ctx = MasContext(sc, make_config(sc, levels=2, K=8))
    v = ctx.vec()
    st = _abi.lib().pncg_subspace_step_noalloc(ctx.h, _ptr(v), _ptr(v), None, _ptr(v), _ptr(v), _ptr(v), 1,
                                                _ptr(ctx.out))
    assert st == 2  # MAS_ERR_STATE
    ctx.close()
    torch.cuda.synchronize()
