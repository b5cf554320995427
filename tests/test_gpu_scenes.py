"""Per-scene iteration of the batched form (several independent scenes in
one context): the per-scene 2x2 steps (pncg_subspace_step_scenes) and
energies (mas_energy_grad_scenes) against the oracle applied to each
scene's own vertices, contacts and update columns (FP64, 1e-10), and the
per-scene driver lowering every scene's energy and gradient."""
import numpy as np
import pytest

from oracle import fem, pncg, woodbury
from paper_2604_19892_amd import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _batch():
    sc, offs = synth.batch_scene(n_scenes=3, size_range=(5e3, 1.2e4), contact_range=(1e3, 3e3))
    d = synth.pool_distance(sc.pool, sc.x)
    act = (d > 0) & (d < sc.dhat)
    base = synth.contact_set(sc.pool['key'][act], sc.pool['idx'][act], sc.pool['grad'][act], d[act])
    curr = synth.churn_set(np.random.default_rng(4), sc, base, 0.3)
    return sc, offs, base, curr


def test_scene_steps_and_energies_match_oracle():
    import torch
    from paper_2604_19892_amd.binding import MasContext, make_config
    print("\n[scenes case] 3 scenes, per-scene 2x2 steps and energies", flush=True)
    sc, offs, base, curr = _batch()
    S = len(offs) - 1
    prob = fem.Problem(sc)
    H = prob.assemble(sc.x, base)
    dS, u, _ = woodbury.classify(prob, base, curr)
    U = woodbury.global_U(prob, curr, u, dS)
    Ht = (H + U @ U.T).tocsr()
    ctx = MasContext(sc, make_config(sc, levels=3, K=8, block_prec="f64"), scene_offsets=offs)
    try:
        n, voff = ctx.scenes()
        assert n == S and np.array_equal(voff, offs)
        ctx.build(ctx.to_lib(sc.x), ctx.contacts(base))
        ctx.woodbury_update(ctx.contacts(curr))
        rng = np.random.default_rng(6)
        g, z, zp, p = rng.standard_normal((4, 3 * sc.N))
        restart = np.array([0, 1, 0], np.int32)
        dp, dvp = ctx.to_lib(p), ctx.to_lib(H @ p)
        out = torch.zeros(S * ctx.out.numel(), dtype=torch.float64, device="cuda")
        ctx.subspace_step_scenes(ctx.to_lib(g), ctx.to_lib(z), ctx.to_lib(zp), ctx.to_lib(H @ z), dp, dvp,
                                 torch.as_tensor(restart, device="cuda"), out)
        o = out.cpu()
        pg = ctx.from_lib(dp)
        for s in range(S):
            dofs = np.arange(3 * offs[s], 3 * offs[s + 1])

            def Hmul(v):
                full = np.zeros(3 * sc.N)
                full[dofs] = v
                return (Ht @ full)[dofs]

            mu, nu, pn, fb, *_ = pncg.subspace_step(g[dofs], z[dofs], p[dofs], Hmul, bool(restart[s]))
            r = pncg.restart_ratio(g[dofs], zp[dofs], z[dofs])
            st = ctx.step_out(o[s * ctx.out.numel():(s + 1) * ctx.out.numel()])
            assert st["mu"] == pytest.approx(mu, rel=1e-10), s
            assert st["nu"] == pytest.approx(nu, rel=1e-10, abs=1e-12 * abs(mu)), s
            assert st["r"] == pytest.approx(r, rel=1e-10), s
            assert st["restart_used"] == restart[s]
            assert rel(pg[dofs], pn) < 1e-10, s
        # per-scene energies at a displaced point
        xt = fem.inertial_target(sc.x, sc.v, sc.h, sc.gravity).reshape(-1)
        x = (sc.x + 1e-4 * rng.standard_normal(sc.x.shape)).reshape(-1)
        dcur = ctx.contacts(curr)
        E = torch.zeros(S, dtype=torch.float64, device="cuda")
        gl = ctx.vec()
        ctx.energy_grad_scenes(ctx.to_lib(x), ctx.to_lib(xt), dcur, E, gl)
        E = E.cpu().numpy()
        tets = np.asarray(sc.tets, np.int64)
        cs = np.searchsorted(offs, curr['idx'][:, 0], side="right") - 1
        for s in range(S):
            vs = slice(offs[s], offs[s + 1])
            dx = x.reshape(-1, 3)[vs] - xt.reshape(-1, 3)[vs]
            Ein = 0.5 * float(np.sum(prob.mass[vs, None] * dx * dx))
            ts = (tets[:, 0] >= offs[s]) & (tets[:, 0] < offs[s + 1])
            Eel = sc.h ** 2 * fem.elastic_energy(x.reshape(-1, 3), tets[ts], prob.Dm_inv[ts], prob.vol[ts],
                                                 prob.mu[ts], prob.lam[ts])
            b, _, _ = fem.barrier(curr['d'][cs == s], sc.dhat)
            assert E[s] == pytest.approx(Ein + Eel + sc.kappa * float(np.sum(b)), rel=1e-10), s
        assert rel(ctx.from_lib(gl), prob.gradient(x, xt, curr)) < 1e-10
        code, msg = ctx.sync()
        assert code == 0, msg
    finally:
        ctx.close()


def test_scene_driver_lowers_every_scene():
    from paper_2604_19892_amd.pncg import ScenePNCG
    print("\n[scenes case] 3 scenes, 30 iterations of the per-scene driver", flush=True)
    sc, offs = synth.batch_scene(n_scenes=3, size_range=(5e3, 1.2e4), contact_range=(1e3, 3e3))
    s = ScenePNCG(sc, offs, block_prec="f32", hess_prec="f32", K=24, levels=3)
    E0 = s.E_host.copy()
    for _ in range(30):
        s.iterate()
    code, msg = s.ctx.sync()
    assert code == 0, msg
    E = np.array([r["E"] for r in s.log])
    assert np.all(np.diff(np.vstack([E0, E]), axis=0) <= 1e-15 * np.abs(E0))
    gn = np.array([r["gnorm"] for r in s.log])
    print("gradient ratios", gn[-1] / gn[0], "builds", s.n_builds, flush=True)
    assert np.all(gn[-1] < 0.1 * gn[0])
    rs = np.array([r["restart"] for r in s.log])
    assert np.any(rs.any(axis=1) & ~rs.all(axis=1))     # scenes restart on their own
    s.ctx.close()
