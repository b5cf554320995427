"""Algorithm 1 on geometric contacts (ComputeConstraintSet at the head of
each iteration, contact keys from the pairs' primitives, ConservativeCCD
for the per-subdomain steps) on the GPU against the oracle's loop
(``oracle.solver.OracleGeoPNCG``).

The stacked-boxes scene: two 10x10x5 boxes half dhat apart, the upper one
falling onto the lower.  Both sides run in float64 from the same state; the
first iterations agree step by step (restart decisions, mu, nu, the number
of contacts and candidates, the step scale, positions).  A longer GPU run
then keeps every surface pair apart and the energy decreasing."""
import numpy as np
import pytest

from oracle import constraint_set as CS
from oracle import contact as C
from oracle.solver import OracleGeoPNCG
from paper_2604_19892_amd import synth

pytestmark = pytest.mark.gpu

EDGE = 1.0 / 9


def test_geometric_iterations_match_oracle():
    import torch
    from paper_2604_19892_amd.pncg import GeoPNCG
    print("\n[geometric case] stacked boxes 10x10x5, 6 iterations against the oracle", flush=True)
    sc = synth.stacked_boxes_scene()
    surf = synth.surface(sc.tets)
    radius = 0.25 * EDGE
    ora = OracleGeoPNCG(sc, surf, radius)
    gpu = GeoPNCG(sc, radius, block_prec="f64", hess_prec="f64")
    dx_prev = 0.0  # ||x_gpu - x_oracle|| at the point the iteration starts from
    for k in range(6):
        ora.iterate()
        gpu.iterate()
        lo, lg = ora.log[-1], gpu.log[-1]
        print("iteration %d: restart %s/%s mu %.6g/%.6g contacts %d/%d candidates %d/%d" % (
            k, lo["restart"], lg["restart"], lo["mu"], lg["mu"], lo["m"], lg["m"], lo["candidates"],
            lg["candidates"]), flush=True)
        assert lo["restart"] == lg["restart"], k
        assert lo["m"] == lg["m"] and lo["candidates"] == lg["candidates"], k
        assert lg["mu"] == pytest.approx(lo["mu"], rel=1e-7), k
        assert lg["nu"] == pytest.approx(lo["nu"], rel=1e-6, abs=1e-9), k
        assert lg["scale"] == lo["scale"] and lg["accepted"] == lo["accepted"], k
        # E at the start point: to first order its difference is bounded by
        # ||grad E|| times the distance between the two start points (the
        # fast mode's float atomics make the trajectories drift apart at
        # rounding level); twice that, plus rounding of E itself
        assert abs(lg["E"] - lo["E"]) <= 2.0 * lo["gnorm"] * dx_prev + 1e-12 * abs(lo["E"]), k
        xg = gpu.ctx.from_lib(gpu.x)
        dx_prev = float(np.linalg.norm(xg - ora.x))
        err = dx_prev / np.linalg.norm(ora.x - sc.x.reshape(-1))
        assert err < 1e-6, (k, err)
    code, msg = gpu.ctx.sync()
    assert code == 0, msg
    gpu.ctx.close()
    torch.cuda.empty_cache()


def test_geometric_run_keeps_surfaces_apart():
    """Forty iterations of float32-block MAS-PNCG on geometric contacts: the
    energy never increases, no surface pair closes (brute force over every
    pair within the candidate radius at the end, oracle distances), and the
    gradient falls."""
    import torch
    from paper_2604_19892_amd.pncg import GeoPNCG
    print("\n[geometric case] stacked boxes 10x10x5, 40 iterations", flush=True)
    sc = synth.stacked_boxes_scene()
    verts, tris, edges = synth.surface(sc.tets)
    radius = 0.25 * EDGE
    gpu = GeoPNCG(sc, radius, block_prec="f32", hess_prec="f32")
    E = [gpu.E_host]
    for _ in range(40):
        gpu.iterate()
        E.append(gpu.E_host)
    code, msg = gpu.ctx.sync()
    assert code == 0, msg
    assert all(b <= a for a, b in zip(E, E[1:]))
    assert gpu.log[-1]["gnorm"] < 1e-2 * gpu.log[0]["gnorm"]
    x = gpu.ctx.from_lib(gpu.x).reshape(-1, 3)
    pairs, kinds, d = CS.constraint_set(x, verts, tris, edges, radius)
    assert len(pairs) > 0 and np.min(d) > 0.0
    print("restarts %d of 40, smallest surface distance %.3e, contacts %d" % (
        gpu.n_restarts, float(np.min(d)), gpu.C.m), flush=True)
    gpu.ctx.close()
    torch.cuda.empty_cache()
