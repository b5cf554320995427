"""The device-resident PNCG iteration against the oracle's Algorithm 1 loop.

Both run the grid scene in float64 from the same state: the first
iterations must agree step by step (mu, nu, restart decisions, positions),
and both must reach ||grad E|| <= 1e-6 ||grad E_0||.
"""
import numpy as np
import pytest

from oracle.solver import OraclePNCG
from paper_2604_19892_amd import synth

pytestmark = pytest.mark.gpu


def test_pncg_trajectory_matches_oracle():
    from paper_2604_19892_amd.pncg import PNCG
    sc = synth.grid_scene()
    ora = OraclePNCG(sc)
    gpu = PNCG(sc, block_prec="f64")
    for k in range(8):
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


@pytest.mark.parametrize("update,rule,precond", [("freeze", "subspace", "mas"), ("rebuild", "subspace", "mas"),
                                                 ("woodbury", "fr", "mas"), ("woodbury", "cd", "mas"),
                                                 ("woodbury", "dk", "mas"), ("rebuild", "dk", "mas"),
                                                 ("woodbury", "subspace", "bj3"), ("woodbury", "fr", "bj3")])
def test_ablation_variants_match_oracle(update, rule, precond):
    """The update strategies and direction rules of the ablation study
    against the oracle's loop with the same variant (ratio test off, so that
    every iteration after the first uses the variant's update and rule)."""
    from paper_2604_19892_amd.pncg import PNCG
    print("\n[ablation case] grid, update %s, rule %s, preconditioner %s" % (update, rule, precond), flush=True)
    sc = synth.grid_scene()
    ora = OraclePNCG(sc, update=update, rule=rule, precond=precond, delta=1e3)
    gpu = PNCG(sc, block_prec="f64", update=update, rule=rule, precond=precond, delta=1e3)
    for k in range(4):
        ora.iterate()
        gpu.iterate()
        lo, lg = ora.log[-1], gpu.log[-1]
        assert lo["restart"] == lg["restart"], k
        assert lo["fallback"] == lg["fallback"], k
        assert lg["mu"] == pytest.approx(lo["mu"], rel=1e-7), k
        assert lg["nu"] == pytest.approx(lo["nu"], rel=1e-6, abs=1e-9), k
        xg = gpu.ctx.from_lib(gpu.x)
        err = np.linalg.norm(xg - ora.x) / np.linalg.norm(ora.x - sc.x.reshape(-1))
        assert err < 1e-6, (k, err)
    assert sum(not r["restart"] for r in gpu.log) == 3
    code, msg = gpu.ctx.sync()
    assert code == 0, msg


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_pncg_reaches_tolerance(prec):
    from paper_2604_19892_amd.pncg import PNCG
    sc = synth.grid_scene()
    gpu = PNCG(sc, block_prec=prec)
    it, secs, rel = gpu.solve(rel_tol=1e-6, max_iter=200)
    print("grid %s: %d iterations, %.3f s, %d restarts" % (prec, it, secs, gpu.n_restarts))
    assert it < 200
    assert rel <= 1e-6
    # the library's norm of the gradient the last iteration started from
    assert gpu.log[-1]["gnorm"] <= 1e-6 * gpu.g0norm * 1.0000001


def test_next_frame_and_later_time_steps():
    """mas_next_frame against implicit Euler written out (v = (x1 - x0)/h,
    x~ = x1 + h v + h^2 g), and three time steps of the two-box scene in a
    row, each solved to 1e-6 of its first gradient with finite energies."""
    import torch
    from oracle import fem
    from paper_2604_19892_amd.pncg import PNCG
    sc = synth.two_boxes_scene(active_frac=0.8)
    s = PNCG(sc, block_prec="f32", hess_prec="f32")
    x0 = s.ctx.from_lib(s.x)
    for f in range(3):
        it, secs, rel = s.solve(rel_tol=1e-6, max_iter=600)
        print("two boxes, time step %d: %d iterations, %d restarts so far" % (f, it, s.n_restarts))
        assert rel <= 1e-6, (f, rel)
        assert np.isfinite(s.E_host)
        x1 = s.ctx.from_lib(s.x)
        s.next_frame()
        v = (x1 - x0) / sc.h
        xt = fem.inertial_target(x1.reshape(-1, 3), v.reshape(-1, 3), sc.h, sc.gravity).reshape(-1)
        assert np.allclose(s.ctx.from_lib(s.v_frame), v, rtol=1e-13, atol=1e-13 * np.abs(v).max())
        assert np.allclose(s.ctx.from_lib(s.xt), xt, rtol=1e-14, atol=1e-14 * np.abs(xt).max())
        x0 = x1
    code, msg = s.ctx.sync()
    assert code == 0, msg
    s.ctx.close()
    torch.cuda.empty_cache()
