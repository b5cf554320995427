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
