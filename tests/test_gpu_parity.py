"""GPU parity: every C ABI call against the FP64 oracle on the same inputs.

Cases: the 8x8x8 grid scene (512 vertices, 16 subdomains, two levels,
scripted update touching every classification branch) and the two stacked
boxes (64,000 vertices, 2,000 subdomains, three levels, 30% scripted churn).
Tolerances: relative 1e-10 (float64 storage), 1e-5 (float32 blocks), 2e-2
(bfloat16 / float16 blocks); integer results (Morton order, Top-K
selection) are compared exactly.
"""
import numpy as np
import pytest

from oracle import fem, mas, pncg, woodbury
from paper_2604_19892_amd import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


class Case:
    """Oracle results and a GPU context for one scene and update."""

    def __init__(self, scene, base, curr, levels, K, block_prec="f64"):
        import torch
        from paper_2604_19892_amd.binding import MasContext, make_config
        self.scene, self.base, self.curr = scene, base, curr
        prob = fem.Problem(scene)
        hier = mas.Hierarchy(scene.X, levels)
        self.prob, self.hier = prob, hier
        self.H = prob.assemble(scene.x, base)
        self.M = mas.MAS(hier, self.H)
        self.dS, self.u, self.case = woodbury.classify(prob, base, curr)
        self.sel = woodbury.topk(hier, curr, self.dS, self.u, K)
        self.blocks = woodbury.updated_blocks(hier, self.H, curr, self.u, self.sel)
        self.U = woodbury.global_U(prob, curr, self.u, self.dS)
        self.ctx = MasContext(scene, make_config(scene, levels=levels, K=K, block_prec=block_prec))
        self.x = self.ctx.to_lib(scene.x)
        self.dbase = self.ctx.contacts(base)
        self.dcurr = self.ctx.contacts(curr)
        self.ctx.build(self.x, self.dbase)
        self.ctx.woodbury_update(self.dcurr)
        code, msg = self.ctx.sync()
        assert code == 0, msg
        self.torch = torch


def grid_case(block_prec="f64"):
    sc = synth.grid_scene()
    base, curr = synth.grid_update_sets(sc)
    return Case(sc, base, curr, levels=2, K=8, block_prec=block_prec)


def boxes_case():
    sc = synth.two_boxes_scene()
    rng = np.random.default_rng(5)
    d = synth.pool_distance(sc.pool, sc.x)
    base = synth.contact_set(sc.pool['key'], sc.pool['idx'], sc.pool['grad'], d)
    curr = synth.churn_set(rng, sc, base, 0.3)
    return Case(sc, base, curr, levels=3, K=8)


@pytest.fixture(scope="module", params=["grid", "boxes"])
def case(request):
    print("\n[parity case] %s" % request.param, flush=True)
    c = grid_case() if request.param == "grid" else boxes_case()
    yield c
    c.ctx.close()


def test_morton_order_matches_oracle(case):
    np.testing.assert_array_equal(case.ctx.perm, case.hier.perm)


def test_level0_blocks(case):
    D = case.hier.num_subdomains(0)
    ds = range(D) if D <= 64 else np.random.default_rng(0).choice(D, 64, replace=False)
    worst = 0.0
    for d in ds:
        Bo = case.M.fine[d]
        n = Bo.shape[0]
        # build state is still in effect for the blocks (the update does not change them)
        Bg = case.ctx.get_block(0, d)[:n, :n]
        worst = max(worst, rel(Bg, Bo))
    assert worst < 1e-10, worst


def test_coarse_blocks(case):
    for l in range(1, case.hier.L):
        _, _, invs = case.M.coarse[l - 1]
        for d, (dofs, Minv) in enumerate(invs):
            n = Minv.shape[0]
            Bg = case.ctx.get_block(l, d)[:n, :n]
            assert rel(Bg, Minv) < 1e-10, (l, d, rel(Bg, Minv))


def test_topk_selection_exact(case):
    rank, sel = case.ctx.get_selection()
    D = case.hier.num_subdomains(0)
    for d in range(D):
        want = case.sel.get(d, [])
        assert rank[d] == len(want), d
        assert list(sel[d, :rank[d]]) == list(want), d
    # every classification branch is exercised
    assert {woodbury.NEW, woodbury.ROTATED, woodbury.STIFFEN, woodbury.SOFTEN} <= set(case.case.tolist())


def test_apply_with_woodbury_update(case):
    rng = np.random.default_rng(1)
    g = rng.standard_normal(3 * case.scene.N)
    zo = case.M.apply(g, case.blocks)
    zg = case.ctx.from_lib(case.ctx.apply(case.ctx.to_lib(g)))
    assert rel(zg, zo) < 1e-10, rel(zg, zo)


def test_apply_symmetric_positive(case):
    rng = np.random.default_rng(2)
    a, b = rng.standard_normal((2, 3 * case.scene.N))
    ctx = case.ctx
    Pa = ctx.from_lib(ctx.apply(ctx.to_lib(a)))
    Pb = ctx.from_lib(ctx.apply(ctx.to_lib(b)))
    assert abs(a @ Pb - b @ Pa) < 1e-11 * abs(a @ Pa)
    assert a @ Pa > 0 and b @ Pb > 0


def test_hess_vec(case):
    rng = np.random.default_rng(3)
    v = rng.standard_normal(3 * case.scene.N)
    yo = case.H @ v
    yo_u = yo + case.U @ (case.U.T @ v)
    ctx = case.ctx
    y0 = ctx.from_lib(ctx.hess_vec(ctx.to_lib(v), with_update=False))
    y1 = ctx.from_lib(ctx.hess_vec(ctx.to_lib(v), with_update=True))
    assert rel(y0, yo) < 1e-10, rel(y0, yo)
    assert rel(y1, yo_u) < 1e-10, rel(y1, yo_u)


def test_subspace_step(case):
    rng = np.random.default_rng(4)
    n = 3 * case.scene.N
    xt = fem.inertial_target(case.scene.x, case.scene.v, case.scene.h, case.scene.gravity).reshape(-1)
    g = case.prob.gradient(case.scene.x, xt, case.curr)
    z = case.M.apply(g, case.blocks)
    z_prev = z + 0.3 * rng.standard_normal(n) * np.abs(z).max()
    p = -0.7 * z_prev + 0.1 * rng.standard_normal(n) * np.abs(z).max()

    def Ht(v):
        return case.H @ v + case.U @ (case.U.T @ v)

    mu, nu, pn, fb, A11, A12, A22 = pncg.subspace_step(g, z, p, Ht, restart=False)
    r = pncg.restart_ratio(g, z_prev, z)
    ctx = case.ctx
    dp = ctx.to_lib(p)
    dvp = ctx.to_lib(case.H @ p)
    out = ctx.subspace_step(ctx.to_lib(g), ctx.to_lib(z), ctx.to_lib(z_prev), ctx.to_lib(case.H @ z), dp, dvp,
                            restart=False)
    s = ctx.step_out()
    assert s['fallback'] == int(fb)
    assert s['mu'] == pytest.approx(mu, rel=1e-10)
    assert s['nu'] == pytest.approx(nu, rel=1e-10, abs=1e-12 * abs(mu))
    assert s['A11'] == pytest.approx(A11, rel=1e-10)
    assert s['A12'] == pytest.approx(A12, rel=1e-10, abs=1e-12 * A11)
    assert s['A22'] == pytest.approx(A22, rel=1e-10)
    assert s['r'] == pytest.approx(r, rel=1e-10)
    assert s['restart_next'] == int(r > 0.3)
    assert rel(ctx.from_lib(dp), pn) < 1e-10
    assert rel(ctx.from_lib(dvp), case.H @ pn) < 1e-10
    # restart form: mu = g.z / z^T H~ z, nu = 0
    mu0, nu0, pn0, fb0, *_ = pncg.subspace_step(g, z, p, Ht, restart=True)
    dp = ctx.to_lib(p)
    dvp = ctx.to_lib(case.H @ p)
    ctx.subspace_step(ctx.to_lib(g), ctx.to_lib(z), None, ctx.to_lib(case.H @ z), dp, dvp, restart=True)
    s = ctx.step_out()
    assert s['mu'] == pytest.approx(mu0, rel=1e-10) and s['nu'] == 0.0 and s['restart_used'] == 1
    assert rel(ctx.from_lib(dp), pn0) < 1e-10


@pytest.mark.parametrize("rule", ["fr", "cd", "dk"])
def test_beta_step(case, rule):
    """pncg_beta_step against the oracle's comparison rules: beta, alpha,
    the new direction and its H_base product, the step, and the restart
    form."""
    from oracle.solver import RULES
    rng = np.random.default_rng(7)
    n = 3 * case.scene.N
    xt = fem.inertial_target(case.scene.x, case.scene.v, case.scene.h, case.scene.gravity).reshape(-1)
    g = case.prob.gradient(case.scene.x, xt, case.curr)
    z = case.M.apply(g, case.blocks)
    sc_z = np.abs(z).max()
    g_prev = g + 0.5 * rng.standard_normal(n) * np.abs(g).max()
    z_prev = case.M.apply(g_prev, case.blocks)
    d_prev = -0.8 * z_prev + 0.05 * rng.standard_normal(n) * sc_z

    def Ht(v):
        return case.H @ v + case.U @ (case.U.T @ v)

    a, b, dn, pn, fb = pncg.beta_step(RULES[rule], g, g_prev, z, z_prev, d_prev, Ht, restart=False)
    assert not fb and b != 0.0
    r = pncg.restart_ratio(g, z_prev, z)
    ctx = case.ctx
    dd, dvd, dp = ctx.to_lib(d_prev), ctx.to_lib(case.H @ d_prev), ctx.vec()
    ctx.beta_step(rule, ctx.to_lib(g), ctx.to_lib(g_prev), ctx.to_lib(z), ctx.to_lib(z_prev),
                  ctx.to_lib(case.H @ z), dd, dvd, False, dp)
    s = ctx.step_out()
    assert s['fallback'] == 0 and s['restart_used'] == 0
    assert s['nu'] == pytest.approx(b, rel=1e-10)
    assert s['mu'] == pytest.approx(a, rel=1e-10)
    assert s['r'] == pytest.approx(r, rel=1e-10)
    assert rel(ctx.from_lib(dd), dn) < 1e-10
    assert rel(ctx.from_lib(dvd), case.H @ dn) < 1e-10
    assert rel(ctx.from_lib(dp), pn) < 1e-10
    # restart form (g_prev not read): the subspace step's restart step
    a0, b0, dn0, pn0, fb0 = pncg.beta_step(RULES[rule], g, None, z, None, None, Ht, restart=True)
    dd, dvd = ctx.to_lib(d_prev), ctx.to_lib(case.H @ d_prev)
    ctx.beta_step(rule, ctx.to_lib(g), None, ctx.to_lib(z), None, ctx.to_lib(case.H @ z), dd, dvd, True, dp)
    s = ctx.step_out()
    assert s['mu'] == pytest.approx(a0, rel=1e-10) and s['nu'] == 0.0 and s['restart_used'] == 1
    assert rel(ctx.from_lib(dp), pn0) < 1e-10
    assert rel(ctx.from_lib(dd), -z) < 1e-15
    # a previous direction pointing uphill: fallback to d = -z
    up = ctx.to_lib(z_prev)
    ctx.beta_step("cd", ctx.to_lib(g), ctx.to_lib(g_prev), ctx.to_lib(z), ctx.to_lib(z_prev),
                  ctx.to_lib(case.H @ z), up, ctx.to_lib(case.H @ z_prev), False, dp)
    s = ctx.step_out()
    a1, b1, dn1, pn1, fb1 = pncg.beta_step(pncg.BETA_CD, g, g_prev, z, z_prev, z_prev, Ht, restart=False)
    assert fb1 and s['fallback'] == 1 and s['nu'] == 0.0
    assert rel(ctx.from_lib(dp), pn1) < 1e-10
    with pytest.raises(Exception):
        ctx.beta_step("fr", ctx.to_lib(g), None, ctx.to_lib(z), None, ctx.to_lib(case.H @ z), dd, dvd, False, dp)


def test_block_jacobi_preconditioner(case):
    """precond = MAS_PRECOND_BJ3: z = blockdiag(H~_ii)^-1 g after mas_build
    (H~ = H_base) and after mas_woodbury_update (H~ = H_base + U U^T),
    against the oracle's dense 3x3 inverses; the MAS block queries refuse."""
    from oracle import jacobi
    from paper_2604_19892_amd.binding import MasContext, make_config
    sc = case.scene
    ctx = MasContext(sc, make_config(sc, levels=case.hier.L, K=8, precond="bj3"))
    try:
        rng = np.random.default_rng(9)
        g = rng.standard_normal(3 * sc.N)
        ctx.build(ctx.to_lib(sc.x), ctx.contacts(case.base))
        z = ctx.from_lib(ctx.apply(ctx.to_lib(g)))
        assert rel(z, jacobi.apply(jacobi.inverse_blocks(case.H), g)) < 1e-12
        hist = case.torch.zeros(9, dtype=case.torch.int32, device="cuda")
        ctx.woodbury_update(ctx.contacts(case.curr), hist)
        z = ctx.from_lib(ctx.apply(ctx.to_lib(g)))
        Ht = case.H + case.U @ case.U.T
        assert rel(z, jacobi.apply(jacobi.inverse_blocks(Ht), g)) < 1e-12
        # hess_vec and the update columns are those of the MAS mode
        v = rng.standard_normal(3 * sc.N)
        y = ctx.from_lib(ctx.hess_vec(ctx.to_lib(v), with_update=True))
        assert rel(y, Ht @ v) < 1e-10
        assert int(hist[0].item()) == int(case.ctx.nsub[0]) and int(hist[1:].sum().item()) == 0
        code, msg = ctx.sync()
        assert code == 0, msg
        with pytest.raises(Exception):
            ctx.get_block(0, 0)
    finally:
        ctx.close()


def test_energy_gradient(case):
    sc = case.scene
    xt = fem.inertial_target(sc.x, sc.v, sc.h, sc.gravity).reshape(-1)
    Eo = case.prob.energy(sc.x, xt, case.curr)
    go = case.prob.gradient(sc.x, xt, case.curr)
    ctx = case.ctx
    dxt = ctx.inertial_target(ctx.to_lib(sc.x), ctx.to_lib(sc.v))
    assert rel(ctx.from_lib(dxt), xt) < 1e-15
    E = case.torch.zeros(1, dtype=case.torch.float64, device="cuda")
    g = ctx.vec()
    ctx.energy_grad(case.x, dxt, case.dcurr, E, g)
    assert float(E.item()) == pytest.approx(Eo, rel=1e-10)
    assert rel(ctx.from_lib(g), go) < 1e-10


def test_stencil_distance_and_safe_step(case):
    sc = case.scene
    ctx = case.ctx
    pool = ctx.contacts(sc.pool)
    ctx.stencil_distance(case.x, pool)
    do = synth.pool_distance(sc.pool, sc.x)
    # d = n . x - off cancels: compare against the size of the summed terms
    scale = np.abs(sc.pool['grad']).sum(1) * np.abs(sc.x).max() + np.abs(sc.pool['off'])
    assert np.all(np.abs(pool.d.cpu().numpy() - do) <= 1e-15 * scale)
    # the step rule itself is compared on identical distances
    pool.d.copy_(case.torch.as_tensor(do, device="cuda"))
    rng = np.random.default_rng(6)
    p = 0.05 * rng.standard_normal(3 * sc.N) * (sc.X.max() - sc.X.min()) / 8
    ao = pncg.safe_alpha(case.hier, sc.pool['idx'], sc.pool['grad'], do, p)
    alpha = case.torch.zeros(case.hier.num_subdomains(0), dtype=case.torch.float64, device="cuda")
    xo = ctx.vec()
    ctx.safe_step(case.x, ctx.to_lib(p), pool, 1.0, xo, alpha)
    assert np.any(ao < 1)
    np.testing.assert_allclose(alpha.cpu().numpy(), ao, rtol=1e-12)
    xn = pncg.step_positions(case.hier, sc.x.reshape(-1), p, ao)
    assert rel(ctx.from_lib(xo), xn) < 1e-14
    # the step-size histogram of the counters
    st = ctx.stats()
    hist = np.zeros(8, np.int64)
    for a in ao:
        hist[0 if a >= 1 else next((i for i in range(1, 7) if a >= 2.0 ** -i), 7)] += 1
    assert st['alpha_hist'] == hist.tolist()
    assert st['safe_left'] == 0
    # halved step reuses the step sizes
    ctx.safe_step(case.x, ctx.to_lib(p), None, 0.5, xo)
    assert rel(ctx.from_lib(xo), pncg.step_positions(case.hier, sc.x.reshape(-1), p, 0.5 * ao)) < 1e-14


def test_safe_step_fallback_when_rounds_do_not_separate(case):
    """A stencil across two subdomains with no net closing rate but one
    vertex closing fast, beside a stencil holding one subdomain to a small
    step: 16 damping rounds cannot separate it at d = 1e-9, and every
    subdomain takes the bound for any mix of steps (oracle: the same
    rule)."""
    sc, hier = case.scene, case.hier
    r = hier.rank
    va = int(np.flatnonzero(r // 32 == 0)[0])
    vb, vb2 = (int(v) for v in np.flatnonzero(r // 32 == 1)[:2])
    idx = np.array([[va, vb, -1, -1], [vb2, -1, -1, -1]], np.int32)
    grad = np.zeros((2, 12))
    grad[0, 2], grad[0, 5], grad[1, 2] = 1.0, -1.0, 1.0
    d = np.array([1e-9, 1e-3])
    p = np.zeros(3 * sc.N)
    p[[3 * va + 2, 3 * vb + 2, 3 * vb2 + 2]] = -1.0
    cset = synth.contact_set(np.array([1, 2], np.uint64), idx, grad, d)
    ao = pncg.safe_alpha(hier, idx, grad, d, p)
    assert ao[0] == pytest.approx(0.9e-9)
    ctx = case.ctx
    alpha = case.torch.zeros(hier.num_subdomains(0), dtype=case.torch.float64, device="cuda")
    xo = ctx.vec()
    ctx.safe_step(case.x, ctx.to_lib(p), ctx.contacts(cset), 1.0, xo, alpha)
    np.testing.assert_allclose(alpha.cpu().numpy(), ao, rtol=1e-12)
    assert ctx.stats()['safe_left'] > 0
    code, msg = ctx.sync()
    assert code == 0, msg


def test_apply_after_rebuild_without_update(case):
    ctx = case.ctx
    ctx.build(case.x, case.dbase)
    rng = np.random.default_rng(7)
    g = rng.standard_normal(3 * case.scene.N)
    zg = ctx.from_lib(ctx.apply(ctx.to_lib(g)))
    assert rel(zg, case.M.apply(g)) < 1e-10
    rank, _ = ctx.get_selection()
    assert np.all(rank == 0)
    ctx.woodbury_update(case.dcurr)      # restore the updated state
    code, msg = ctx.sync()
    assert code == 0, msg


_ORACLE = {}


def oracle_case(name):
    """The oracle side of a parity case (no GPU context), cached per scene."""
    if name not in _ORACLE:
        if name == "grid":
            sc = synth.grid_scene()
            base, curr = synth.grid_update_sets(sc)
            L = 2
        else:
            sc = synth.two_boxes_scene()
            rng = np.random.default_rng(5)
            d = synth.pool_distance(sc.pool, sc.x)
            base = synth.contact_set(sc.pool['key'], sc.pool['idx'], sc.pool['grad'], d)
            curr = synth.churn_set(rng, sc, base, 0.3)
            L = 3
        c = Case.__new__(Case)
        c.scene, c.base, c.curr = sc, base, curr
        c.prob = fem.Problem(sc)
        c.hier = mas.Hierarchy(sc.X, L)
        c.H = c.prob.assemble(sc.x, base)
        c.M = mas.MAS(c.hier, c.H)
        c.dS, c.u, c.case = woodbury.classify(c.prob, base, curr)
        c.sel = woodbury.topk(c.hier, curr, c.dS, c.u, 8)
        c.blocks = woodbury.updated_blocks(c.hier, c.H, curr, c.u, c.sel)
        c.U = woodbury.global_U(c.prob, curr, c.u, c.dS)
        _ORACLE[name] = (c, L)
    return _ORACLE[name]


# (scene, storage, guard, tolerance, least share of blocks stored as asked):
# guard 0 never promotes, so every block is stored in the requested 16-bit
# format; the default guard keeps most two-box blocks in 16 bits and
# promotes the stiff grid blocks (the share is then only reported).
LOW = [("grid", "f32", 0.5, 1e-5, 1.0), ("grid", "bf16", 0.0, 2e-2, 1.0), ("grid", "f16", 0.0, 2e-2, 1.0),
       ("grid", "bf16", 0.5, 2e-2, 0.0), ("boxes", "bf16", 0.5, 2e-2, 0.8), ("boxes", "f16", 0.5, 2e-2, 0.95)]


@pytest.mark.parametrize("name,prec,guard,tol,share", LOW)
def test_low_precision_blocks(name, prec, guard, tol, share):
    from paper_2604_19892_amd.binding import MasContext, make_config
    print("\n[parity case] %s %s guard %g" % (name, prec, guard), flush=True)
    c, L = oracle_case(name)
    ctx = MasContext(c.scene, make_config(c.scene, levels=L, K=8, block_prec=prec, prec_guard=guard))
    ctx.build(ctx.to_lib(c.scene.x), ctx.contacts(c.base))
    ctx.woodbury_update(ctx.contacts(c.curr))
    code, msg = ctx.sync()
    assert code == 0, msg
    counts = ctx.block_precisions(0)
    D = c.hier.num_subdomains(0)
    print("stored block precisions", counts)
    assert sum(counts.values()) == D
    assert counts[prec] >= share * D, counts
    if guard == 0.0:
        assert counts[prec] == D
    rng = np.random.default_rng(8)
    g = rng.standard_normal(3 * c.scene.N)
    zo = c.M.apply(g, c.blocks)
    zg = ctx.from_lib(ctx.apply(ctx.to_lib(g)))
    err = rel(zg, zo)
    print("apply rel err %s: %.3e (%d of %d blocks stored as %s)" % (prec, err, counts[prec], D, prec))
    assert err < tol
    # Hessian snapshot in float32 for the mixed forms
    v = rng.standard_normal(3 * c.scene.N)
    yo = c.H @ v + c.U @ (c.U.T @ v)
    y = ctx.from_lib(ctx.hess_vec(ctx.to_lib(v), with_update=True))
    assert rel(y, yo) < 1e-5
    ctx.close()


def test_nonfinite_inputs_are_reported(case):
    """A NaN in g (mas_apply) or an inf in v (hess_vec) sets
    MAS_ERR_NONFINITE, which the read clears."""
    ctx = case.ctx
    n = 3 * case.scene.N
    g = np.ones(n)
    g[n // 3] = np.nan
    ctx.apply(ctx.to_lib(g))
    code, msg = ctx.sync()
    assert code == 6, (code, msg)
    assert ctx.sync()[0] == 0
    v = np.ones(n)
    v[-1] = np.inf
    ctx.hess_vec(ctx.to_lib(v), with_update=False)
    code, msg = ctx.sync()
    assert code == 6, (code, msg)
    assert ctx.sync()[0] == 0


def test_capacity_limits():
    """Contact sets beyond max_contacts are refused before any launch."""
    from paper_2604_19892_amd._abi import MasError
    from paper_2604_19892_amd.binding import MasContext, make_config
    print("\n[parity case] grid with max_contacts 100", flush=True)
    sc = synth.grid_scene()
    base, curr = synth.grid_update_sets(sc)
    assert base['key'].size > 100 and curr['key'].size > 100
    ctx = MasContext(sc, make_config(sc, levels=2, K=8, max_contacts=100))
    with pytest.raises(MasError) as e:
        ctx.build(ctx.to_lib(sc.x), ctx.contacts(base))
    assert e.value.code == 1
    small = synth.subset(base, slice(0, 100))
    ctx.build(ctx.to_lib(sc.x), ctx.contacts(small))
    with pytest.raises(MasError) as e:
        ctx.woodbury_update(ctx.contacts(curr))
    assert e.value.code == 1
    ctx.woodbury_update(ctx.contacts(synth.subset(curr, slice(0, 100))))
    code, msg = ctx.sync()
    assert code == 0, msg
    ctx.close()


def test_iteration_stats(case):
    """Branch counts of the classification and the kept ranks, against the
    oracle's classification of the same sets."""
    st = case.ctx.stats()
    k = case.prob.contact_stiffness(case.curr['d'])
    act = k > 0
    # a base entry with k = 0 classifies like absence (dS = k either way);
    # the library keeps only base contacts with k > 0 and counts these as new
    kb = case.prob.contact_stiffness(case.base['d'])
    where = {int(q): i for i, q in enumerate(case.base['key'])}
    br = case.case.copy()
    for c_ in np.nonzero(act)[0]:
        b = where.get(int(case.curr['key'][c_]))
        if b is None or kb[b] == 0:
            br[c_] = woodbury.NEW
    assert st['contacts'] == case.curr['key'].size
    assert st['active'] == int(act.sum())
    assert st['n_new'] == int(((br == woodbury.NEW) & act).sum())
    assert st['n_rotated'] == int(((br == woodbury.ROTATED) & act).sum())
    assert st['n_stiffened'] == int(((br == woodbury.STIFFEN) & act).sum())
    assert st['n_softened'] == int(((br == woodbury.SOFTEN) & act).sum())
    ranks = [len(v) for v in case.sel.values()]
    assert st['rank_sum'] == sum(ranks)
    assert st['rank_max'] == max(ranks)


def stiff_case(prec, guard):
    """Grid scene whose contacts sit at d ~ 1e-9 (barrier stiffness ~1e9 x
    the vertex mass): inverse blocks far beyond float32 resolution."""
    import torch
    from paper_2604_19892_amd.binding import MasContext, make_config
    sc = synth.grid_scene()
    base, curr = synth.grid_update_sets(sc)
    base = dict(base)
    curr = dict(curr)
    # stiff contacts only on vertices of the first eight Morton subdomains
    rank = np.empty(sc.N, np.int64)
    rank[mas.morton_perm(sc.X)] = np.arange(sc.N)
    low_b = rank[base['idx'][:, 0]] < 256
    low_c = rank[curr['idx'][:, 0]] < 256
    base['d'] = np.where(low_b, 2e-9, base['d'])
    curr['d'] = np.where(low_c & (curr['d'] < 5e-4), 1e-9, curr['d'])
    case = Case.__new__(Case)
    case.scene, case.base, case.curr = sc, base, curr
    prob = fem.Problem(sc)
    hier = mas.Hierarchy(sc.X, 2)
    case.prob, case.hier = prob, hier
    case.H = prob.assemble(sc.x, base)
    case.M = mas.MAS(hier, case.H)
    case.dS, case.u, case.case = woodbury.classify(prob, base, curr)
    case.sel = woodbury.topk(hier, curr, case.dS, case.u, 8)
    case.blocks = woodbury.updated_blocks(hier, case.H, curr, case.u, case.sel)
    case.ctx = MasContext(sc, make_config(sc, levels=2, K=8, block_prec=prec, prec_guard=guard))
    case.x = case.ctx.to_lib(sc.x)
    case.ctx.build(case.x, case.ctx.contacts(base))
    case.ctx.woodbury_update(case.ctx.contacts(curr))
    case.torch = torch
    return case


def test_stiff_blocks_are_promoted_and_stay_definite():
    print("\n[parity case] grid stiff f32 guarded", flush=True)
    c = stiff_case("f32", 0.5)
    code, msg = c.ctx.sync()
    assert code == 0, msg
    counts = c.ctx.block_precisions(0)
    print("stored block precisions", counts)
    assert counts["f64"] > 0 and counts["f32"] > 0
    rng = np.random.default_rng(9)
    g = rng.standard_normal(3 * c.scene.N)
    zo = c.M.apply(g, c.blocks)
    zg = c.ctx.from_lib(c.ctx.apply(c.ctx.to_lib(g)))
    assert rel(zg, zo) < 1e-5, rel(zg, zo)
    a = rng.standard_normal(3 * c.scene.N)
    Pa = c.ctx.from_lib(c.ctx.apply(c.ctx.to_lib(a)))
    assert a @ Pa > 0
    c.ctx.close()


def test_indefinite_block_is_reported():
    """Negative vertex masses make the level-0 blocks indefinite: the build
    must flag MAS_ERR_NOT_SPD with the failing block named, not fault."""
    import dataclasses
    from paper_2604_19892_amd.binding import MasContext, make_config
    print("\n[parity case] grid with negative density", flush=True)
    sc = synth.grid_scene()
    sc = dataclasses.replace(sc, density=-1e3 * np.asarray(sc.density))
    base, _ = synth.grid_update_sets(sc)
    ctx = MasContext(sc, make_config(sc, levels=2, K=8))
    ctx.build(ctx.to_lib(sc.x), ctx.contacts(base))
    code, msg = ctx.sync()
    assert code == 5, (code, msg)
    assert "level-0 block" in msg, msg
    # the sticky error is cleared by the read
    assert ctx.sync()[0] == 0
    ctx.close()
