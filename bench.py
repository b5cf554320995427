#!/usr/bin/env python
"""MAS-PNCG iterations per second on one MI355X.

Workload: eight spiky soft balls (the Puffer Balls shape: 1.14M vertices,
2.71M tets, 1.25M affine contact stencils of which ~1M start active, four
MAS levels, Top-K 8), float32 level-0 blocks and element Hessians, float64
vectors, barrier sums, capacitance factors and 2x2 solve.  One step is one
full PNCG iteration of Algorithm 1 (contact distances, RebuildMAS or the
Woodbury update, z = P g, H_base z, the subspace step, safe steps, trial
energy/gradient with the descent check, restart test); restarts happen
when the restart test asks for them, inside the timed region.

Prints one JSON line.  The timed steps run in blocks of ten iterations,
each block from the scene's start (x^0, a restart), so that about 1M
contacts are active through them.  The roofline object covers the level-0
kernel of mas_apply, timed with HIP events recorded by the library on its
own stream during the timed steps.  ``warm_frame`` times iterations of a
later time step (the first two solved to tolerance first).  After the timed steps, ``tol_solve`` solves from
the same start to ||grad E|| <= 1e-6 ||grad E_0|| five times per level-0
block storage (f64 with float64 element Hessians; f32, bf16 and f16 with
float32 element Hessians) and reports iterations and wall-clock times.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PNCG iters/s + mas_apply HBM GB/s at 1.1M verts; mixed vs FP64 at same ‖∇E‖ tol"
HBM_PEAK_GBS = 8000.0
PK = 96 * 97 // 2


def apply_l0_bytes(ctx, counts, hist):
    """Algorithmic bytes of one level-0 apply launch: every block in its
    stored precision (+ row scales for 16-bit), g read, z written, coarse
    corrections read, ranks, and per updated subdomain its float64 W, slot
    columns and capacitance factor."""
    N = ctx.N
    D0 = int(ctx.nsub[0])
    size = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}
    b = sum(n * (PK * size[p] + (96 * 4 if size[p] == 2 else 0)) for p, n in counts.items())
    b += 2 * 8 * 3 * N
    nodes = N
    for _ in range(1, ctx.levels):
        nodes = -(-nodes // 32)
        b += 8 * 3 * nodes
    b += 4 * D0
    for r, cnt in enumerate(hist):
        if r:
            b += cnt * (96 * r * 8 + r * 112 + 8 * r * (r + 1) // 2)
    return b


def hv_bytes(ctx, hess_prec, n_active):
    """Algorithmic bytes of one Hessian-vector launch: every tet's snapshot
    (45 tangent + 9 Dm^-1 entries in the Hessian storage precision) and its
    four vertex indices once, every active base stencil's column (12 doubles)
    and indices once, the lumped masses, v read and y written."""
    sH = 8 if hess_prec == "f64" else 4
    N = ctx.N
    return ctx.scene.T * (54 * sH + 16) + n_active * (12 * 8 + 16) + 8 * N + 2 * 8 * 3 * N


def update_bytes(ctx, solver, rec, hist):
    """Algorithmic bytes of one mas_woodbury_update call: every current
    contact's key, indices, distance and gradient read and its dS and
    indices written; for each active one its base entry looked up (key-table
    slot, k, base gradient); for each contact with dS > 0 its u column
    written and its candidate entry written and read; per updated subdomain
    its stored block read once (the mean stored size), its float64 W, slot
    columns and capacitance factor written; ranks written and read."""
    size = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}
    counts = solver.precision_counts
    D0 = int(ctx.nsub[0])
    m, act = rec["contacts"], rec["active"]
    nu = rec["n_new"] + rec["n_rotated"] + rec["n_stiffened"]
    b = m * (8 + 16 + 8 + 96) + m * (8 + 16)
    b += act * (12 + 8 + 96)
    b += nu * (96 + 2 * 4)
    blk = sum(n * (PK * size[p] + (96 * 4 if size[p] == 2 else 0)) for p, n in counts.items()) / max(D0, 1)
    for r, cnt in enumerate(hist):
        if r:
            b += cnt * (blk + 96 * r * 8 + r * 112 + 8 * r * (r + 1) // 2)
    return b + 2 * 4 * D0


def warm_frame(sc, prec, hess_prec, iters, tol=1e-6, max_iter=800):
    """A later time step: the first two are solved to ||grad E|| <= tol
    ||grad E_0|| (untimed; implicit Euler between them), then `iters`
    iterations of the third are timed, started from the second's end, the
    regime of a running simulation (contacts near their balance)."""
    import numpy as np
    import torch
    from paper_2604_19892_amd.pncg import PNCG
    s = PNCG(sc, block_prec=prec, hess_prec=hess_prec)
    frames = []
    for _ in range(2):
        it, sec, rel = s.solve(rel_tol=tol, max_iter=max_iter)
        frames.append({"iters": it, "seconds": sec, "rel_gnorm": rel, "converged": bool(rel <= tol)})
        s.next_frame()
    def active():
        return int(((s.pool.d > 0) & (s.pool.d < sc.dhat)).sum().item())

    a0 = active()
    r0 = s.n_restarts
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(iters):
        s.iterate()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    code, msg = s.ctx.sync()
    out = {"iters_per_s": iters / dt, "ms_per_iter": 1e3 * dt / iters, "iters": iters,
           "restart_fraction": (s.n_restarts - r0) / iters,
           "active_contacts_first_last": [a0, active()],
           "previous_frames": frames, "status": code}
    s.ctx.close()
    del s
    torch.cuda.empty_cache()
    return out


def geometric_measure(iters=20, warmup=3):
    """Algorithm 1 on geometric contacts (GeoPNCG): the stacked-boxes scene
    at 2 x 40x40x20 vertices, the upper box falling onto the lower; per
    iteration ComputeConstraintSet at x (contacts) and within the candidate
    radius (CCD), the trial point's set for the descent check, the CCD safe
    step.  Iterations per second over ``iters`` timed iterations and the
    library's stage times (from as many further iterations with the
    timers on)."""
    import numpy as np
    import torch
    from paper_2604_19892_amd import synth
    from paper_2604_19892_amd.pncg import GeoPNCG
    sc = synth.stacked_boxes_scene(nxy=40, nz=20, levels=3)
    edge = 1.0 / 39
    g = GeoPNCG(sc, 0.25 * edge, block_prec="f32", hess_prec="f32")
    for _ in range(warmup):
        g.iterate()
    ctx = g.ctx
    r0, k0 = g.n_restarts, len(g.log)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(iters):
        g.iterate()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    # stage times from as many further iterations with every timer on
    ctx.profile(True)
    for _ in range(iters):
        g.iterate()
    stages = {k: ctx.profile_read(k)[0] / iters for k in ("build", "update", "apply", "hess_vec", "energy",
                                                          "subspace", "ccd", "constraint_set")}
    ctx.profile(False)
    code, msg = ctx.sync()
    recs = g.log[k0:k0 + iters]
    out = {"workload": "stacked boxes 2 x 40x40x20 (%d verts, %d tets), upper box falling at 0.5 m/s" % (sc.N, sc.T),
           "iters_per_s": iters / dt, "ms_per_iter": 1e3 * dt / iters, "iters": iters,
           "restart_fraction": sum(1 for r in recs if r["restart"]) / iters,
           "contacts_mean": float(np.mean([r["m"] for r in recs])),
           "ccd_candidates_mean": float(np.mean([r["candidates"] for r in recs])),
           "descent_halvings": int(sum(1 for r in recs if r["scale"] < 1.0)),
           "stage_ms_per_iter": stages, "status": code}
    ctx.close()
    del g
    torch.cuda.empty_cache()
    return out


BLOCK = 10

TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SRC = {"k_apply_l0": "k_apply.hip", "k_hv_range": "k_hessvec.hip"}


def _src_hash(kernel):
    """Hash of the kernel's source file and of the shared layout header."""
    h = hashlib.sha256()
    for name in (KERNEL_SRC[kernel], "common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2604_19892_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def traffic_record(kernel, prec, workload):
    """Measured HBM bytes per launch of a kernel from rocprofv3 counters, if
    they were taken on the kernel's current source and this workload."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    rec = json.load(open(TRAFFIC_JSON)).get(kernel)
    if not rec or rec.get("source_sha256") != _src_hash(kernel):
        return None
    if rec.get("prec") != prec or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")


def traffic_from_counters(fetch_dir, write_dir, prec, workload):
    """Writes profiles/traffic.json from two rocprofv3 --pmc runs of
    `bench.py --copy-probe` (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).
    Each counter is scaled by what it reads for the 1 GiB device copy of the
    probe (known size) and averaged over the kernel's dispatches."""
    import csv
    import glob
    import numpy as np

    def per_kernel(d, counter):
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        vals = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals

    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        vals = per_kernel(d, counter)
        copy = max(v for k, vs in vals.items() if "copyBuffer" in k for v in vs)
        scale = (1 << 30) / (copy * 1024.0)
        for kern in KERNEL_SRC:
            vs = [v for k, v_ in vals.items() if kern in k for v in v_]
            if vs:
                e = out.setdefault(kern, {"prec": prec, "workload": workload, "source_sha256": _src_hash(kern)})
                e[counter.lower() + "_bytes"] = float(np.mean(vs)) * 1024.0 * scale
                e[counter.lower() + "_scale"] = scale
                e["dispatches"] = len(vs)
    for e in out.values():
        e["bytes_per_launch"] = e.get("fetch_size_bytes", 0.0) + e.get("write_size_bytes", 0.0)
    json.dump(out, open(TRAFFIC_JSON, "w"), indent=1)
    print(json.dumps(out, indent=1))


def cpu_baseline(full_N, iters=3):
    """The FP64 oracle (Algorithm 1 with full-rebuild semantics) on a
    bounded sample of the same workload family, scaled linearly in vertex
    count to the full scene."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle.solver import OraclePNCG
    from paper_2604_19892_amd import synth
    sc = synth.puffer_scene(core=(12, 12, 13), n_spikes=130, spike_len=7, pool_size=46000)
    s = OraclePNCG(sc)
    t = time.perf_counter()
    for _ in range(iters):
        s.iterate()
    dt = time.perf_counter() - t
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": iters / dt * sc.N / full_N, "unit": "iters/s", "cores": int(threads),
            "kind": "oracle", "extrapolated": True,
            "sample": "%d oracle iterations (first one a restart) on an 8-ball puffer scene with %d vertices, "
                      "%d tets, %d stencils; %.1f s; iters/s extrapolated linearly in vertex count by %d/%d"
                      % (iters, sc.N, sc.T, sc.pool['key'].size, dt, sc.N, full_N)}


def hbm_probe(reps=5):
    """Plain device copy and sum of 1 GiB with torch's own kernels, timed with
    events on torch's stream: what simple streaming kernels reach on this
    GPU, reported beside the nominal 8 TB/s."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    a.sum()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    for _ in range(reps):
        a.sum()
    e2.record()
    torch.cuda.synchronize()
    gib = float(1 << 30)
    out = {"copy_GBps": reps * 2 * gib / (e0.elapsed_time(e1) * 1e-3) / 1e9,
           "read_GBps": reps * gib / (e1.elapsed_time(e2) * 1e-3) / 1e9, "bytes": int(gib)}
    del a, b
    torch.cuda.empty_cache()
    return out


def ccd_measure(ctx, solver, reps=10):
    """Conservative CCD (supplement Section 3.4) of every point-triangle /
    edge-edge stencil of the pool along the step to the inertial target
    x~ - x (the time step's predicted motion), timed with the library's
    events; the inputs are device tensors prepared before the clock."""
    import torch
    pool = solver.pool
    m = int(pool.idx.shape[0])
    step = solver.xt - solver.x
    kind = ((pool.key >> 60) == 3).to(torch.uint8)          # key tag 3: edge-edge, 2: point-triangle
    dist = pool.d.clamp_min(0.0)
    ap = torch.empty(m, dtype=torch.float64, device=pool.idx.device)
    alpha = torch.empty(int(ctx.nsub[0]), dtype=torch.float64, device=pool.idx.device)
    ctx.ccd_steps(solver.x, step, pool.idx, kind, dist, ap, alpha)
    ctx.profile(True)
    for _ in range(reps):
        ctx.ccd_steps(solver.x, step, pool.idx, kind, dist, ap, alpha)
    ms, n = ctx.profile_read("ccd")
    ctx.profile(False)
    us = 1e3 * ms / max(n, 1)
    return {"pairs": m, "us_per_call": us, "pairs_per_s": m / (us * 1e-6),
            "pairs_with_step_below_1": float((ap < 1.0).double().mean().item()),
            "subdomains_with_step_below_1": float((alpha < 1.0).double().mean().item())}


def contact_measure(ctx, solver, dhat, reps=10):
    """Contact narrow phase (distance, n = grad d and closest-feature type)
    of every point-triangle / edge-edge stencil of the pool at the current
    positions, timed with the library's events.  Algorithmic bytes per
    pair: the four vertex ids and the kind read, the distance, twelve
    gradient entries and the type written, and four vertex positions
    gathered (counted once per pair)."""
    import torch
    pool = solver.pool
    m = int(pool.idx.shape[0])
    dev = pool.idx.device
    kind = ((pool.key >> 60) == 3).to(torch.uint8)          # key tag 3: edge-edge, 2: point-triangle
    dist = torch.empty(m, dtype=torch.float64, device=dev)
    grad = torch.empty(m, 12, dtype=torch.float64, device=dev)
    ty = torch.empty(m, dtype=torch.uint8, device=dev)
    ctx.contact_distances(solver.x, pool.idx, kind, dist, grad, ty)
    ctx.profile(True)
    for _ in range(reps):
        ctx.contact_distances(solver.x, pool.idx, kind, dist, grad, ty)
    ms, n = ctx.profile_read("contact")
    ctx.profile(False)
    us = 1e3 * ms / max(n, 1)
    per_pair = 16 + 1 + 4 * 24 + 8 + 12 * 8 + 1
    return {"pairs": m, "us_per_call": us, "pairs_per_s": m / (us * 1e-6),
            "algorithmic_GB_per_s": per_pair * m / (us * 1e-6) / 1e9, "bytes_per_pair": per_pair,
            "pairs_below_dhat": float((dist < dhat).double().mean().item())}


def constraint_set_measure(ctx, sc, x, reps=5):
    """ComputeConstraintSet (mas_constraint_set) over the scene's whole
    boundary surface at the current positions: hashed-grid broad phase and
    narrow phase, timed with the library's events around the whole call
    (which includes its two host read-backs).  The first call, which sizes
    the grid tables, is not timed."""
    import numpy as np
    import torch
    from paper_2604_19892_amd import synth
    verts, tris, edges = synth.surface(sc.tets)
    dev = x.device
    r = ctx.rank
    vt = torch.as_tensor(r[verts].astype(np.int32), device=dev)
    tt = torch.as_tensor(r[tris].astype(np.int32), device=dev)
    et = torch.as_tensor(r[edges].astype(np.int32), device=dev)
    cap = 1 << 22
    pairs = torch.empty(cap, 4, dtype=torch.int32, device=dev)
    kind = torch.empty(cap, dtype=torch.uint8, device=dev)
    dist = torch.empty(cap, dtype=torch.float64, device=dev)
    grad = torch.empty(cap, 12, dtype=torch.float64, device=dev)
    n = ctx.constraint_set(x, vt, tt, et, sc.dhat, pairs, kind, dist, grad)
    ctx.profile(True)
    for _ in range(reps):
        n = ctx.constraint_set(x, vt, tt, et, sc.dhat, pairs, kind, dist, grad)
    ms, calls = ctx.profile_read("constraint_set")
    ctx.profile(False)
    k = min(n, cap)
    n_pt = int((kind[:k] == 0).sum().item())
    return {"surface_vertices": int(len(verts)), "surface_triangles": int(len(tris)),
            "surface_edges": int(len(edges)), "dhat": sc.dhat, "pairs": int(n), "pt_pairs": n_pt,
            "ee_pairs": int(k - n_pt), "ms_per_call": ms / max(calls, 1)}


# block storage forms of the tolerance solves: (requested level-0 storage,
# element Hessian storage, precision guard; None = the library's default)
SOLVE_FORMS = {"f64": ("f64", "f64", None), "f32": ("f32", "f32", None), "bf16": ("bf16", "f32", None),
               "f16": ("f16", "f32", None), "bf16_all": ("bf16", "f32", 0.0), "f16_all": ("f16", "f32", 0.0)}


def tolerance_solves(sc, forms, tol, max_iter, repeats):
    """PNCG solves per storage form from the same start to ||grad E|| <=
    tol ||grad E_0||: iterations and wall-clock seconds of each, and the
    level-0 blocks actually stored in each precision (the guard promotes
    blocks whose conditioning the requested format cannot hold; the *_all
    forms switch it off).  One context per form, reset to the start before
    each of ``repeats`` solves (its blocks are rebuilt at the first
    iteration).  Trajectories differ between runs (float64 sums taken
    through atomics in no fixed order, restart decisions near the
    threshold), so the spread is reported beside the means."""
    import numpy as np
    import torch
    from paper_2604_19892_amd.pncg import PNCG
    runs = {f: [] for f in forms}
    stored = {}
    for f in forms:
        bp, hp, guard = SOLVE_FORMS[f]
        s = PNCG(sc, block_prec=bp, hess_prec=hp, prec_guard=guard)
        # with the guard off the stiff blocks lose definiteness in 16 bits
        # (capacitance pivots <= 0) and the solve does not converge: one
        # short run shows it
        reps, cap = (1, min(max_iter, 300)) if guard == 0.0 else (repeats, max_iter)
        for _ in range(reps):
            s.reset()
            it, sec, rel = s.solve(rel_tol=tol, max_iter=cap)
            code, msg = s.ctx.sync()
            runs[f].append({"iters": it, "seconds": sec, "rel_gnorm": rel, "converged": bool(rel <= tol),
                            "status": code})
            print("[bench] solve %s: %d iters %.2fs rel %.2e" % (f, it, sec, rel), file=sys.stderr, flush=True)
        stored[f] = s.ctx.block_precisions(0)   # the last rebuild's storage
        s.ctx.close()
        del s
        torch.cuda.empty_cache()
    out = {"tol": tol, "max_iter": max_iter, "repeats": repeats, "runs": runs, "stored_level0_blocks": stored,
           "forms": {f: {"block_storage": SOLVE_FORMS[f][0], "hessian_storage": SOLVE_FORMS[f][1],
                         "guard": "off" if SOLVE_FORMS[f][2] == 0.0 else "default"} for f in forms},
           "seconds": {}, "iters": {}, "mean_ms_per_iter": {}}
    for f, rs in runs.items():
        if all(r["converged"] for r in rs):
            t = np.array([r["seconds"] for r in rs])
            n = np.array([r["iters"] for r in rs])
            out["seconds"][f] = {"mean": float(t.mean()), "min": float(t.min()), "max": float(t.max()),
                                 "median": float(np.median(t))}
            out["iters"][f] = {"mean": float(n.mean()), "min": int(n.min()), "max": int(n.max())}
            out["mean_ms_per_iter"][f] = 1e3 * float(t.sum() / n.sum())
    if "f64" in out["seconds"]:
        f64 = out["seconds"]["f64"]
        out["f64_seconds_over"] = {f: {"mean": f64["mean"] / v["mean"], "median": f64["median"] / v["median"]}
                                   for f, v in out["seconds"].items() if f != "f64"}
        ms64 = out["mean_ms_per_iter"]["f64"]
        out["f64_ms_per_iter_over"] = {f: ms64 / v for f, v in out["mean_ms_per_iter"].items() if f != "f64"}
    return out


ABLATION_VARIANTS = (("woodbury", "subspace", "mas"), ("freeze", "subspace", "mas"),
                     ("rebuild", "subspace", "mas"), ("woodbury", "fr", "mas"), ("woodbury", "cd", "mas"),
                     ("woodbury", "dk", "mas"), ("woodbury", "subspace", "bj3"))


def _variant_solve(sc, update, rule, precond, tol, max_iter, prec="f32", hierarchy="morton"):
    import torch
    from paper_2604_19892_amd.pncg import PNCG
    s = PNCG(sc, block_prec=prec, hess_prec="f32", update=update, rule=rule, precond=precond, hierarchy=hierarchy)
    it, sec, rel = s.solve(rel_tol=tol, max_iter=max_iter)
    code, msg = s.ctx.sync()
    rec = {"update": update, "rule": rule, "preconditioner": precond, "hierarchy": hierarchy, "iters": it,
           "seconds": sec, "ms_per_iter": 1e3 * sec / max(it, 1), "rel_gnorm": rel, "converged": bool(rel <= tol),
           "restarts": s.n_restarts, "status": code}
    s.ctx.close()
    del s
    torch.cuda.empty_cache()
    return rec


def ablation_solves(sc, tol, max_iter):
    """The ablation study's variants on one scene (Section 5): update
    strategy (Woodbury, Freeze, Full Rebuild), direction rule (2x2 subspace
    step, FR, CD, DK) and preconditioner (MAS, 3x3 block-Jacobi); one solve
    each from the scene's start to ||grad E|| <= tol ||grad E_0|| (at most
    max_iter iterations)."""
    runs = []
    for update, rule, precond in ABLATION_VARIANTS:
        rec = _variant_solve(sc, update, rule, precond, tol, max_iter)
        print("[bench] ablation %s/%s/%s: %d iters %.2fs rel %.2e" % (
            update, rule, precond, rec["iters"], rec["seconds"], rec["rel_gnorm"]), file=sys.stderr, flush=True)
        runs.append(rec)
    return {"workload": sc.name, "tol": tol, "max_iter": max_iter, "block_storage": "f32",
            "hessian_storage": "f32", "runs": runs}


def hierarchy_solves(sc, tol, max_iter, repeats=2):
    """MAS on the Morton order against the connectivity-aware hierarchy
    (supplement Section 1.2, with the stencils active at the start as
    reconnection links) on the same scene: solves from the start to tol
    ||grad E_0||, and how many level-0 subdomains hold vertices of more than
    one body in each order."""
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    from paper_2604_19892_amd import synth
    from paper_2604_19892_amd.binding import vertex_order
    t = np.asarray(sc.tets, np.int64)
    A = sp.coo_matrix((np.ones(t.size * 4), (np.repeat(t, 4, axis=1).ravel(), np.tile(t, (1, 4)).ravel())),
                      shape=(sc.N, sc.N)).tocsr()
    _, lab = connected_components(A, directed=False)
    runs = {}
    for h in ("morton", "connectivity"):
        t0 = time.perf_counter()
        links = synth.contact_links(sc.pool, sc.x, sc.dhat) if h == "connectivity" else None
        perm = vertex_order(sc.X, sc.tets, sc.levels, h, links)
        order_s = time.perf_counter() - t0
        n32 = (sc.N // 32) * 32
        b = lab[perm[:n32]].reshape(-1, 32)
        recs = []
        for _ in range(repeats):
            rec = _variant_solve(sc, "woodbury", "subspace", "mas", tol, max_iter, hierarchy=h)
            print("[bench] hierarchy %s: %d iters %.2fs rel %.2e" % (h, rec["iters"], rec["seconds"],
                                                                    rec["rel_gnorm"]), file=sys.stderr, flush=True)
            recs.append(rec)
        runs[h] = {"solves": recs, "order_seconds_host": order_s,
                   "level0_subdomains_mixing_bodies": int((b.min(1) != b.max(1)).sum()),
                   "level0_subdomains": int(-(-sc.N // 32))}
    return {"workload": sc.name, "tol": tol, "max_iter": max_iter, "block_storage": "f32", "runs": runs}


def batched_measure(steps=30, tol=1e-6, max_iter=600):
    """Many independent scenes in one context (the batched configuration):
    64 stacked-box scenes of 5k..120k vertices and 1k..40k stencils, K = 24,
    three levels; every stage is one launch over all scenes, and each scene
    keeps its own 2x2 step scalars, restart decision and descent check
    (ScenePNCG).  Iterations per second over blocks of ten from the start,
    the Woodbury rank histogram, then a solve until every scene's gradient
    is below tol of its own first one, with the iteration at which each got
    there."""
    import numpy as np
    import torch
    from paper_2604_19892_amd import synth
    from paper_2604_19892_amd.pncg import ScenePNCG
    t0 = time.perf_counter()
    sc, offs = synth.batch_scene()
    gen_s = time.perf_counter() - t0
    s = ScenePNCG(sc, offs, block_prec="f32", hess_prec="f32")
    ctx = s.ctx
    for _ in range(BLOCK):                       # warm-up block
        s.iterate()
    hist = torch.zeros(sc.K + 1, dtype=torch.int64, device="cuda")
    hist += s.rank_hist
    hist.zero_()
    torch.cuda.synchronize()
    dt, done, n_upd, builds0, restarts = 0.0, 0, 0, s.n_builds, 0
    while done < steps:
        s.reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(min(BLOCK, steps - done)):
            any_restart = bool(s.restart.any())
            restarts += int(s.restart.sum())
            s.iterate()
            if not any_restart:
                hist += s.rank_hist
                n_upd += 1
        torch.cuda.synchronize()
        dt += time.perf_counter() - t
        done += BLOCK
    builds = s.n_builds - builds0
    s.reset()
    first, it, sec, rel_end = s.solve(rel_tol=tol, max_iter=max_iter)
    code, msg = ctx.sync()
    sizes = np.diff(offs)
    reached = first[first >= 0]
    out = {"workload": "%d stacked-box scenes, %d..%d verts each (%d verts, %d tets, %d stencils in all)"
                       % (len(sizes), sizes.min(), sizes.max(), sc.N, sc.T, sc.pool['key'].size),
           "levels": int(ctx.levels), "K": int(sc.K), "generation_s": gen_s,
           "iters_per_s": steps / dt, "ms_per_iter": 1e3 * dt / steps,
           "scene_restart_fraction": restarts / (steps * len(sizes)), "iterations_with_a_rebuild": builds / steps,
           "woodbury_rank_hist": hist.cpu().numpy().tolist(),
           "solve": {"iters": it, "seconds": sec, "tol": tol, "scenes_converged": int(reached.size),
                     "scene_iters_to_tol": {"min": int(reached.min()) if reached.size else None,
                                            "median": float(np.median(reached)) if reached.size else None,
                                            "max": int(reached.max()) if reached.size else None},
                     "not_converged": [{"scene": int(q), "verts": int(sizes[q]), "rel_gnorm_end": float(rel_end[q]),
                                        "restarts_last_10": int(sum(r["restart"][q] for r in s.log[-10:]))}
                                       for q in np.nonzero(first < 0)[0]]},
           "per_scene_step_scalars": True, "status": code}
    ctx.close()
    del s
    torch.cuda.empty_cache()
    return out


def stiffness_sweep(tol, max_iter, moduli=(2.15e4, 1e5, 1e6, 1e7)):
    """MAS-PNCG against 3x3 block-Jacobi PNCG as the material stiffens
    (Section 5, stiffness robustness): the two-box scene with one Young's
    modulus per run, and with the modulus graded geometrically over the
    height from 2.15e4 to 1e7 (a 500-fold span).  Barrier stiffness 1e3 rho
    edge^3, as for the puffer balls: with rho edge^3 the stiff materials
    press the stencils to distances where the blocks lose definiteness in
    float64."""
    from paper_2604_19892_amd import synth
    base = synth.two_boxes_scene(active_frac=0.8, kappa_scale=1e3)
    scenes = [(float(E), synth.with_youngs(base, E)) for E in moduli]
    scenes.append(("graded 2.15e4..1e7", synth.graded_stiffness(base)))
    runs = []
    for label, sc in scenes:
        for precond in ("mas", "bj3"):
            rec = _variant_solve(sc, "woodbury", "subspace", precond, tol, max_iter)
            rec["youngs"] = label
            print("[bench] stiffness %s %s: %d iters %.2fs rel %.2e" % (
                label, precond, rec["iters"], rec["seconds"], rec["rel_gnorm"]), file=sys.stderr, flush=True)
            runs.append(rec)
    return {"workload": "two_boxes (64000 verts, 288990 tets, 20000 stencils)", "tol": tol, "max_iter": max_iter,
            "runs": runs}


def precision_errors(sc, seed=12):
    """Error of each output of the mixed-precision forms against the float64
    form on the same inputs at the full scene: mas_apply after a rebuild at
    the start and a Woodbury update with the contacts a quarter of the way
    to the inertial target, and hess_vec with the update, for random g and v
    (relative 2-norm errors).  The float64 form itself matches the oracle to
    1e-10 (parity tests); the stored blocks of each form are listed."""
    import numpy as np
    import torch
    from paper_2604_19892_amd.pncg import PNCG
    rng = np.random.default_rng(seed)
    g0 = rng.standard_normal(3 * sc.N)
    v0 = rng.standard_normal(3 * sc.N)
    outs, stored = {}, {}
    for f in ("f64", "f32", "bf16", "f16", "bf16_all", "f16_all"):
        bp, hp, guard = SOLVE_FORMS[f]
        s = PNCG(sc, block_prec=bp, hess_prec=hp, prec_guard=guard)
        ctx = s.ctx
        ctx.build(s.x, s.pool)
        stored[f] = ctx.block_precisions(0)
        x1 = s.x + 0.25 * (s.xt - s.x)
        ctx.stencil_distance(x1, s.pool_t)
        ctx.woodbury_update(s.pool_t)
        z = ctx.apply(ctx.to_lib(g0))
        y = ctx.hess_vec(ctx.to_lib(v0), with_update=True)
        code, msg = ctx.sync()
        outs[f] = (z.cpu().numpy(), y.cpu().numpy(), code)
        ctx.close()
        del s, ctx
        torch.cuda.empty_cache()
    zr, yr, _ = outs["f64"]
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return {"inputs": "rebuild at the start, update with the contacts at x0 + (x~ - x0) / 4, random g and v",
            "stored_level0_blocks": stored,
            "mas_apply_rel_err": {f: rel(o[0], zr) for f, o in outs.items() if f != "f64"},
            "hess_vec_rel_err": {f: rel(o[1], yr) for f, o in outs.items() if f != "f64"},
            "status": {f: o[2] for f, o in outs.items()},
            "tolerances": {"f32": 1e-5, "bf16": 2e-2, "f16": 2e-2}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", default="f32", choices=["f64", "f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the solves to the gradient tolerance (f64 vs mixed storage)")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-frame regime")
    ap.add_argument("--no-geo", action="store_true", help="skip the geometric-contacts measurement")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the ablation variants and the stiffness sweep")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-scenes measurement")
    ap.add_argument("--solve-tol", type=float, default=1e-6)
    ap.add_argument("--solve-max-iter", type=int, default=1500)
    ap.add_argument("--solve-repeats", type=int, default=5)
    ap.add_argument("--small", action="store_true", help="two-boxes scene instead (quick check)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (reference size for rocprofv3 byte counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc output folders and exit")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from_counters(args.traffic_from[0], args.traffic_from[1], args.prec,
                              "two_boxes" if args.small else "puffer_balls")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (how it would shard is described "
              "in the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2604_19892_amd import synth
    from paper_2604_19892_amd.pncg import PNCG

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    if args.small:
        sc = synth.two_boxes_scene(active_frac=0.8)
        workload = "two_boxes"
    else:
        sc = synth.puffer_scene()
        workload = "puffer_balls"
    print("[bench] scene %s: %d verts %d tets %d stencils (%.1fs)"
          % (workload, sc.N, sc.T, sc.pool['key'].size, time.perf_counter() - t0), file=sys.stderr, flush=True)
    hess_prec = "f64" if args.prec == "f64" else "f32"
    solver = PNCG(sc, block_prec=args.prec, hess_prec=hess_prec)
    ctx = solver.ctx
    print("[bench] context ready (%.1fs)" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    # timed steps: blocks of BLOCK iterations, each from the scene's start
    # (x^0, a restart), so that about 1M contacts stay active through them
    for i in range(args.warmup):
        if i % BLOCK == 0:
            solver.reset()
        solver.iterate()
    torch.cuda.synchronize()
    print("[bench] warmup done (%d iters)" % args.warmup, file=sys.stderr, flush=True)

    solver.track_precisions = True
    if solver.precision_counts is None:
        solver.precision_counts = ctx.block_precisions(0)
    # counters of the same blocks, in an untimed pass (reading them
    # synchronises the stream every iteration), with every stage timer
    timer_names = ("apply_l0", "apply", "hv_tets", "hess_vec", "update", "capacitance", "build", "energy",
                   "subspace")
    stage = {k: 0.0 for k in timer_names}
    ctx.profile(True)
    solver.collect_stats = True
    recs, upd_bytes = [], []
    done = 0
    while done < args.steps:
        solver.reset()
        ctx.profile_read("energy")           # the reset's own energy call is not a step
        for i in range(min(BLOCK, args.steps - done)):
            restart = solver.restart
            solver.iterate()
            recs.append(solver.log[-1])
            if not restart:
                upd_bytes.append(update_bytes(ctx, solver, solver.log[-1],
                                              solver.rank_hist.cpu().numpy().tolist()))
        done += BLOCK
        for k in timer_names:
            stage[k] += ctx.profile_read(k)[0]
    solver.collect_stats = False
    # the timed pass: only the timers of the roofline records (each timed
    # launch adds an event pair to the stream); the rank histograms are
    # summed on the device (no host read), the algorithmic bytes are linear
    # in them
    timed_names = ("apply_l0", "hv_tets", "update")
    ctx.profile(True, timers=timed_names)
    hist_acc = torch.zeros_like(solver.rank_hist, dtype=torch.int64)
    # the sum's kernel is loaded on its first call: not inside the timed region
    hist_acc += solver.rank_hist
    hist_acc.zero_()
    torch.cuda.synchronize()
    r0 = solver.n_restarts
    n_upd = 0
    timers = {k: [0.0, 0] for k in timed_names}
    dt = 0.0
    done = 0
    while done < args.steps:
        solver.reset()
        n = min(BLOCK, args.steps - done)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(n):
            restart = solver.restart
            solver.iterate()
            if not restart:
                hist_acc += solver.rank_hist
                n_upd += 1
        torch.cuda.synchronize()
        dt += time.perf_counter() - t
        done += n
        for k in timed_names:
            ms, cnt = ctx.profile_read(k)
            timers[k][0] += ms
            timers[k][1] += cnt
    restarts = solver.n_restarts - r0
    ctx.profile(False)
    print("[bench] timed %d iters in %.3fs" % (args.steps, dt), file=sys.stderr, flush=True)
    hist_sum = hist_acc.cpu().numpy().tolist()
    # per apply launch: the mean of the per-step bytes (linear in the
    # histogram of the step; restarts carry no update)
    zero = apply_l0_bytes(ctx, solver.precision_counts, [0])
    with_upd = apply_l0_bytes(ctx, solver.precision_counts, hist_sum) - zero
    l0_mean = zero + with_upd / args.steps
    l0_bytes = [l0_mean] * args.steps

    ms_l0, n_l0 = timers["apply_l0"]
    bytes_l0 = l0_bytes
    achieved = sum(bytes_l0) / (ms_l0 * 1e-3) / 1e9 if n_l0 else 0.0
    ms_hv, n_hv = timers["hv_tets"]
    actives = [r["active_pool"] for r in recs]
    n_active = int(np.mean(actives))
    hv_b = hv_bytes(ctx, hess_prec, n_active)
    hv_achieved = n_hv * hv_b / (ms_hv * 1e-3) / 1e9 if n_hv else 0.0
    ms_up, n_up = timers["update"]
    up_mean = float(np.mean(upd_bytes)) if upd_bytes else 0.0
    up_achieved = n_up * up_mean / (ms_up * 1e-3) / 1e9 if n_up else 0.0
    traffic = traffic_record("k_apply_l0", args.prec, workload)
    traffic_hv = traffic_record("k_hv_range", args.prec, workload)
    if args.copy_probe:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    alpha_hist = [sum(r["alpha_hist"][q] for r in recs) for q in range(8)]

    out = {
        "metric": METRIC,
        "value": args.steps / dt,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "vertices": int(sc.N), "tets": int(sc.T), "stencils": int(sc.pool['key'].size),
            "levels": int(ctx.levels), "K": int(ctx.cfg.max_rank),
            "arithmetic": "f64 (vectors, barrier sums, capacitance, 2x2 solve; products with stored blocks "
                          "accumulate in f64)",
            "block_storage": args.prec, "hessian_storage": hess_prec,
            "timed_steps": "blocks of %d iterations, each from the scene's start (x^0, a restart)" % BLOCK,
            "restarts_in_timed_steps": int(restarts),
            "stored_block_precisions": solver.precision_counts,
        },
        "active_contacts_per_step": {"mean": float(np.mean(actives)), "min": int(min(actives)),
                                     "max": int(max(actives))},
        "restart_fraction": restarts / args.steps,
        "counters_pass": "active contacts, step sizes, fallbacks, update bytes: an untimed pass over the same "
                         "blocks with per-iteration counters",
        "alpha_hist_subdomains": {"bins": "[0] alpha = 1, [i] alpha in [2^-i, 2^(1-i)) for i = 1..6, [7] < 2^-6",
                                  "counts": alpha_hist},
        "safe_step_fallbacks": int(sum(1 for r in recs if r["safe_left"] > 0)),
        "descent_halvings": int(sum(1 for r in recs if r["scale"] < 1.0)),
        "mas_apply_GBps": achieved,
        "roofline": {
            "kernel": "k_apply_l0 (level-0 blocks + Woodbury correction of mas_apply)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "bytes_per_launch": float(np.mean(bytes_l0)) if bytes_l0 else 0.0,
            "launches": int(n_l0), "avg_us": 1e3 * ms_l0 / max(n_l0, 1),
        },
        "roofline_hess_vec": {
            "kernel": "k_hv_range (tets, base stencils and mass of hess_vec)", "bound": "hbm",
            "achieved": hv_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hv_achieved / HBM_PEAK_GBS,
            "traffic": traffic_hv, "bytes_per_launch": hv_b, "active_base_stencils": n_active,
            "launches": int(n_hv), "avg_us": 1e3 * ms_hv / max(n_hv, 1),
        },
        "roofline_woodbury_update": {
            "call": "mas_woodbury_update (classification, Top-K, capacitance; all its launches)",
            "bound": "hbm", "achieved": up_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": up_achieved / HBM_PEAK_GBS,
            "bytes_per_call": up_mean,
            "calls": int(n_up), "avg_us": 1e3 * ms_up / max(n_up, 1),
        },
        "stage_ms_per_step": {k: v / args.steps for k, v in stage.items()},
        "stage_timers": "HIP events around each call, from the counters pass over the same blocks (the timed "
                        "pass records only k_apply_l0, k_hv_range and the update call)",
        "woodbury_rank_hist": hist_sum,
        "gnorm_rel": solver.log[-1]["gnorm"] / solver.g0norm if solver.g0norm else None,
    }
    code, msg = ctx.sync()
    if code != 0:
        print("[bench] library error: %s" % msg, file=sys.stderr)
        sys.exit(1)
    out["ccd"] = ccd_measure(ctx, solver)
    out["contact_narrow_phase"] = contact_measure(ctx, solver, sc.dhat)
    out["constraint_set"] = constraint_set_measure(ctx, sc, solver.x)
    out["hbm_probe"] = hbm_probe()
    solver.ctx.close()
    del solver, ctx
    torch.cuda.empty_cache()
    if not args.no_warm:
        print("[bench] warm frame", file=sys.stderr, flush=True)
        out["warm_frame"] = warm_frame(sc, args.prec, hess_prec, 60)
    if not args.no_geo:
        print("[bench] geometric contacts", file=sys.stderr, flush=True)
        out["geometric_contacts"] = geometric_measure()
    if not args.no_solve:
        print("[bench] precision errors", file=sys.stderr, flush=True)
        out["precision_errors"] = precision_errors(sc)
        out["tol_solve"] = tolerance_solves(sc, tuple(SOLVE_FORMS), args.solve_tol,
                                            args.solve_max_iter, args.solve_repeats)
    if not args.no_batch:
        print("[bench] batched scenes", file=sys.stderr, flush=True)
        out["batched"] = batched_measure()
    if not args.no_ablation:
        print("[bench] ablations", file=sys.stderr, flush=True)
        out["ablations"] = ablation_solves(sc, args.solve_tol, args.solve_max_iter)
        out["stiffness_sweep"] = stiffness_sweep(args.solve_tol, args.solve_max_iter)
        out["hierarchy"] = hierarchy_solves(sc, args.solve_tol, args.solve_max_iter)
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sc.N)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
