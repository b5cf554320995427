"""Device-resident MAS-PNCG iteration (Algorithm 1) driven through the C ABI.

Per iteration: contact distances of the affine stencil pool, RebuildMAS or
the Woodbury update, z = P g, v_z = H_base z, the 2x2 subspace step (which
also advances H_base p by linearity), per-subdomain safe steps, the trial
energy and gradient, and the restart decision.  The only host reads per
iteration are the trial energy (descent check) and the step scalars.

The descent check halves every subdomain's step until the energy does not
increase (at most ``max_halvings`` times); if none does, the point is kept
and the next iteration restarts.  The paper does not describe its line
search.
"""
from __future__ import annotations

import contextlib
import time

import numpy as np
import torch

from . import synth
from .binding import DeviceContacts, MasContext, make_config


UPDATES = ("woodbury", "freeze", "rebuild")
RULES = ("subspace", "fr", "cd", "dk")


class PNCG:
    """``update`` and ``rule`` select the variants of the ablation study
    (Section 5): "woodbury" (the method), "freeze" (the restart's MAS kept
    until the next restart: max_rank 0, so the preconditioner takes no
    Top-K columns while H~ keeps the untruncated U) or "rebuild" (mas_build
    at every iteration; H_base p is then recomputed by one more hess_vec);
    "subspace" (the method's 2x2 step) or a comparison rule "fr", "cd",
    "dk" (pncg_beta_step); ``precond`` "bj3" swaps MAS for the 3x3
    block-Jacobi comparison preconditioner; ``hierarchy`` "connectivity"
    builds the MAS levels on the connectivity-aware order."""

    def __init__(self, scene, block_prec="f32", levels=None, K=None, delta=0.3, hess_prec=None,
                 max_halvings=8, device="cuda", deterministic=False, prec_guard=None, collect_stats=False,
                 update="woodbury", rule="subspace", precond="mas", hierarchy="morton", graph=False):
        if update not in UPDATES or rule not in RULES:
            raise ValueError("unknown update strategy or direction rule")
        # graph mode: the device part of each iteration (build or update up
        # to the trial point's energy) is captured once per form and buffer
        # assignment in a HIP graph and replayed; everything runs on a
        # stream of the solver's own
        self.graph = bool(graph)
        self.stream = torch.cuda.Stream() if self.graph else None
        self._graphs = {}
        with self._on_stream():
            self._init(scene, block_prec, levels, K, delta, hess_prec, max_halvings, device, deterministic,
                       prec_guard, collect_stats, update, rule, precond, hierarchy)

    def _on_stream(self):
        return torch.cuda.stream(self.stream) if self.stream is not None else contextlib.nullcontext()

    def _init(self, scene, block_prec, levels, K, delta, hess_prec, max_halvings, device, deterministic,
              prec_guard, collect_stats, update, rule, precond, hierarchy):
        self.update = update
        self.rule = rule
        if update == "freeze":
            K = 0
        cfg = make_config(scene, levels=levels, K=K, block_prec=block_prec, hess_prec=hess_prec,
                          delta=delta, deterministic=deterministic, prec_guard=prec_guard, precond=precond,
                          hierarchy=hierarchy)
        self.precond = precond
        self.hierarchy = hierarchy
        self.collect_stats = collect_stats
        # the connectivity-aware hierarchy links the vertices of the
        # stencils active at the start (its reconnection edges)
        links = synth.contact_links(scene.pool, scene.x, scene.dhat) if hierarchy == "connectivity" else None
        self.ctx = ctx = MasContext(scene, cfg, device=device, links=links)
        self.scene = scene
        self.max_halvings = max_halvings
        self.pool = ctx.contacts(scene.pool, sort=True)
        # a second view of the pool with its own distance array for trial points
        self.pool_t = DeviceContacts.__new__(DeviceContacts)
        self.pool_t.__dict__.update(self.pool.__dict__)
        self.pool_t.d = torch.zeros_like(self.pool.d)
        self.x = ctx.to_lib(scene.x)
        self.x0 = self.x.clone()               # the scene's start
        self.x_frame = self.x.clone()          # x^t of the current time step
        self.v_frame = ctx.to_lib(scene.v)     # v^t
        self.xt = ctx.inertial_target(self.x, self.v_frame)
        v = ctx.vec
        self.x_trial, self.g, self.g_trial = v(), v(), v()
        self.z, self.z_prev, self.vz, self.p, self.vp = v(), v(), v(), v(), v()
        self.step = v() if rule != "subspace" else None
        self.E = torch.zeros(1, dtype=torch.float64, device=device)
        # the trial energy and a copy of the step scalars side by side, so
        # that one read brings both to the host
        self._readback = torch.zeros(1 + ctx.out.numel(), dtype=torch.float64, device=device)
        self.E_trial = self._readback[:1]
        self.rank_hist = torch.zeros(max(cfg.max_rank, 0) + 1, dtype=torch.int32, device=device)
        ctx.stencil_distance(self.x, self.pool)
        ctx.energy_grad(self.x, self.xt, self.pool, self.E, self.g)
        self.E_host = float(self.E.item())
        self.restart = True
        self.k = 0
        self.fk = 0                            # iterations in the current time step
        self.frames = 0
        self.n_restarts = 0
        self.n_halvings = 0
        self.n_rejected = 0
        self.log = []
        self.g0norm = None
        self.track_precisions = False
        self.precision_counts = None

    def _device_part(self, restart, z_prev):
        """The launches of one iteration up to the trial point's energy: no
        host read, no allocation (capturable).  Returns the step vector."""
        ctx = self.ctx
        # p and vp hold the previous step (subspace) or direction (rules) and
        # its H_base product
        if restart:
            ctx.build(self.x, self.pool)
        elif self.update == "rebuild":
            ctx.build(self.x, self.pool)
            ctx.hess_vec(self.p, with_update=False, y=self.vp)
        else:
            ctx.woodbury_update(self.pool, self.rank_hist)
        ctx.apply(self.g, self.z)
        ctx.hess_vec(self.z, with_update=False, y=self.vz)
        if self.rule == "subspace":
            ctx.subspace_step(self.g, self.z, z_prev, self.vz, self.p, self.vp, restart)
            step = self.p
        else:
            # g_trial holds the previous iterate's gradient after an accepted
            # step; a rejected one makes this iteration a restart
            ctx.beta_step(self.rule, self.g, self.g_trial, self.z, z_prev, self.vz, self.p, self.vp,
                          restart, self.step)
            step = self.step
        ctx.safe_step(self.x, step, self.pool, 1.0, self.x_trial)
        ctx.stencil_distance(self.x_trial, self.pool_t)
        ctx.energy_grad(self.x_trial, self.xt, self.pool_t, self.E_trial, self.g_trial)
        return step

    def iterate(self):
        with self._on_stream():
            return self._iterate()

    def _iterate(self):
        ctx = self.ctx
        z_prev = self.z_prev if self.fk > 0 else None
        if self.graph:
            # one graph per form (restart or not, with or without z_prev) and
            # buffer assignment (the swaps below alternate it)
            key = (self.restart, z_prev is None, self.x.data_ptr(), self.z.data_ptr(), self.g.data_ptr(),
                   self.pool.d.data_ptr())
            gr = self._graphs.get(key)
            if gr is None:
                gr = torch.cuda.CUDAGraph()
                with torch.cuda.graph(gr, stream=self.stream):
                    self._device_part(self.restart, z_prev)
                self._graphs[key] = gr
            gr.replay()
            step = self.p if self.rule == "subspace" else self.step
        else:
            step = self._device_part(self.restart, z_prev)
        if self.restart:
            self.n_restarts += 1
            if self.track_precisions:
                self.precision_counts = ctx.block_precisions(0)
        scale = 1.0
        accepted = False
        self._readback[1:].copy_(ctx.out)
        rb = self._readback.cpu()
        st = ctx.step_out(rb[1:])
        for h in range(self.max_halvings + 1):
            if h > 0:
                ctx.stencil_distance(self.x_trial, self.pool_t)
                ctx.energy_grad(self.x_trial, self.xt, self.pool_t, self.E_trial, self.g_trial)
                Et = float(self.E_trial.item())
            else:
                Et = float(rb[0])
            if Et <= self.E_host:
                accepted = True
                break
            if h < self.max_halvings:
                scale *= 0.5
                self.n_halvings += 1
                ctx.safe_step(self.x, step, None, scale, self.x_trial)
        if self.g0norm is None:
            self.g0norm = np.sqrt(st["gnorm2"])
        rec = dict(k=self.k, gnorm=float(np.sqrt(st["gnorm2"])), znorm=float(np.sqrt(st["znorm2"])),
                   mu=st["mu"], nu=st["nu"], r=st["r"], restart=bool(self.restart),
                   fallback=bool(st["fallback"]), E=Et, scale=scale, accepted=accepted)
        if self.collect_stats:
            # counters of this iteration's update (none on a restart) and
            # safe step; reading them synchronises the stream
            rec.update(ctx.stats())
            rec["active_pool"] = int(((self.pool.d > 0) & (self.pool.d < self.scene.dhat)).sum().item())
        self.log.append(rec)
        if accepted:
            self.x, self.x_trial = self.x_trial, self.x
            self.g, self.g_trial = self.g_trial, self.g
            self.pool.d, self.pool_t.d = self.pool_t.d, self.pool.d
            self.z, self.z_prev = self.z_prev, self.z
            self.E_host = Et
            self.restart = bool(st["restart_next"])
        else:
            # no step decreased the energy: stay at x and rebuild the
            # preconditioner there (the next step starts afresh)
            self.z, self.z_prev = self.z_prev, self.z
            self.n_rejected += 1
            self.restart = True
        self.k += 1
        self.fk += 1
        return st

    def reset(self):
        """Back to the scene's start (x^0, v^0, its inertial target); the
        next iteration restarts."""
        with self._on_stream():
            self._reset()

    def _reset(self):
        ctx = self.ctx
        self.x.copy_(self.x0)
        self.x_frame.copy_(self.x0)
        self.v_frame.copy_(ctx.to_lib(self.scene.v))
        ctx.inertial_target(self.x, self.v_frame, self.xt)
        ctx.stencil_distance(self.x, self.pool)
        ctx.energy_grad(self.x, self.xt, self.pool, self.E, self.g)
        self.E_host = float(self.E.item())
        self.restart = True
        self.fk = 0

    def next_frame(self):
        """Ends the time step at the current x (implicit Euler): x^{t+1} = x,
        v^{t+1} = (x - x^t) / h, a new inertial target, and the next
        iteration restarts (Algorithm 1 starts every time step with a
        rebuild)."""
        with self._on_stream():
            self._next_frame()

    def _next_frame(self):
        ctx = self.ctx
        ctx.next_frame(self.x, self.x_frame, self.v_frame, self.xt)
        self.x_frame.copy_(self.x)
        ctx.energy_grad(self.x, self.xt, self.pool, self.E, self.g)
        self.E_host = float(self.E.item())
        self.restart = True
        self.fk = 0
        self.frames += 1

    def gnorm(self):
        with self._on_stream():
            return float(torch.linalg.vector_norm(self.g).item())

    def solve(self, rel_tol=1e-6, max_iter=1000):
        """Iterates until the gradient an iteration starts from satisfies
        ||grad E|| <= rel_tol ||grad E_0|| (norms from the subspace step
        kernel; that last iteration is counted and timed).  Returns
        (iterations, seconds, relative gradient norm)."""
        torch.cuda.synchronize()
        t = time.perf_counter()
        g0 = None
        rel = float("inf")
        it = 0
        while it < max_iter:
            st = self.iterate()
            it += 1
            gn = float(np.sqrt(st["gnorm2"]))
            if g0 is None:
                g0 = gn
            rel = gn / g0 if g0 > 0 else 0.0
            if rel <= rel_tol or not np.isfinite(rel):
                break
        torch.cuda.synchronize()
        return it, time.perf_counter() - t, rel


class ScenePNCG:
    """Algorithm 1 on several independent scenes in one context (the batched
    form): every stage is one launch over all scenes, and each scene keeps
    its own 2x2 step scalars, restart decision, descent check and step
    halving (pncg_subspace_step_scenes, mas_energy_grad_scenes,
    mas_step_scenes).  When any scene restarts, every scene's preconditioner
    is rebuilt (mas_build covers the whole context); the scenes that do not
    restart keep their directions, whose H_base product is then recomputed.
    The host reads the per-scene trial energies and step scalars once per
    iteration (and once per halving round)."""

    def __init__(self, scene, offsets, block_prec="f32", hess_prec=None, levels=None, K=None, delta=0.3,
                 max_halvings=8, device="cuda"):
        cfg = make_config(scene, levels=levels, K=K, block_prec=block_prec, hess_prec=hess_prec, delta=delta)
        self.ctx = ctx = MasContext(scene, cfg, device=device, scene_offsets=offsets)
        self.S, voff = ctx.scenes()
        S = self.S
        self.scene = scene
        self.max_halvings = max_halvings
        self.pool = ctx.contacts(scene.pool, sort=True)
        self.pool_t = DeviceContacts.__new__(DeviceContacts)
        self.pool_t.__dict__.update(self.pool.__dict__)
        self.pool_t.d = torch.zeros_like(self.pool.d)
        self.x = ctx.to_lib(scene.x)
        self.x0 = self.x.clone()
        self.xt = ctx.inertial_target(self.x, ctx.to_lib(scene.v))
        v = ctx.vec
        self.x_trial, self.g, self.g_trial = v(), v(), v()
        self.z, self.z_prev, self.vz, self.p, self.vp = v(), v(), v(), v(), v()
        self.nout = ctx.out.numel()
        self.E = torch.zeros(S, dtype=torch.float64, device=device)
        # per-scene trial energies and step scalars side by side (one read)
        self._readback = torch.zeros(S + S * self.nout, dtype=torch.float64, device=device)
        self.E_trial = self._readback[:S]
        self.out = self._readback[S:]
        self.restart_dev = torch.ones(S, dtype=torch.int32, device=device)
        self.scale_dev = torch.ones(S, dtype=torch.float64, device=device)
        self.rank_hist = torch.zeros(max(cfg.max_rank, 0) + 1, dtype=torch.int32, device=device)
        self.seg_dof = torch.as_tensor(np.repeat(np.repeat(np.arange(S), np.diff(voff)), 3), device=device)
        ctx.stencil_distance(self.x, self.pool)
        ctx.energy_grad_scenes(self.x, self.xt, self.pool, self.E, self.g)
        self.E_host = self.E.cpu().numpy().copy()
        self.restart = np.ones(S, bool)
        self.k = 0
        self.n_builds = 0
        self.log = []

    def reset(self):
        """Back to the scenes' start; the next iteration restarts every scene."""
        self.x = self.x0.clone()
        self.ctx.stencil_distance(self.x, self.pool)
        self.ctx.energy_grad_scenes(self.x, self.xt, self.pool, self.E, self.g)
        self.E_host = self.E.cpu().numpy().copy()
        self.restart = np.ones(self.S, bool)
        self.k = 0

    def solve(self, rel_tol=1e-6, max_iter=1000):
        """Iterates until every scene's gradient satisfies ||g_s|| <= rel_tol
        ||g_s0|| (norms from the step kernel).  Returns the iteration at which
        each scene first did (-1 if not), the iterations, the seconds and
        each scene's final ||g_s|| / ||g_s0||."""
        torch.cuda.synchronize()
        t = time.perf_counter()
        first = -np.ones(self.S, np.int64)
        g0 = None
        it = 0
        gn = None
        while it < max_iter:
            outs = self.iterate()
            it += 1
            gn = np.sqrt([o["gnorm2"] for o in outs])
            if g0 is None:
                g0 = np.maximum(gn, 1e-300)
            done = gn <= rel_tol * g0
            first = np.where((first < 0) & done, it, first)
            if np.all(first >= 0):
                break
        torch.cuda.synchronize()
        return first, it, time.perf_counter() - t, (gn / g0 if gn is not None else None)

    def _outs(self, flat):
        return [self.ctx.step_out(flat[s * self.nout:(s + 1) * self.nout]) for s in range(self.S)]

    def iterate(self):
        ctx = self.ctx
        S = self.S
        if self.restart.any():
            ctx.build(self.x, self.pool)
            self.n_builds += 1
            if not self.restart.all():
                ctx.hess_vec(self.p, with_update=False, y=self.vp)
        else:
            ctx.woodbury_update(self.pool, self.rank_hist)
        ctx.apply(self.g, self.z)
        ctx.hess_vec(self.z, with_update=False, y=self.vz)
        self.restart_dev.copy_(torch.as_tensor(self.restart.astype(np.int32)))
        ctx.subspace_step_scenes(self.g, self.z, self.z_prev if self.k > 0 else None, self.vz, self.p, self.vp,
                                 self.restart_dev, self.out)
        ctx.safe_step(self.x, self.p, self.pool, 1.0, self.x_trial)
        ctx.stencil_distance(self.x_trial, self.pool_t)
        ctx.energy_grad_scenes(self.x_trial, self.xt, self.pool_t, self.E_trial, self.g_trial)
        rb = self._readback.cpu().numpy()
        Et = rb[:S].copy()
        outs = self._outs(rb[S:])
        accepted = Et <= self.E_host
        scale = np.ones(S)
        for _ in range(self.max_halvings):
            if accepted.all():
                break
            scale[~accepted] *= 0.5
            self.scale_dev.copy_(torch.as_tensor(scale))
            ctx.step_scenes(self.x, self.p, self.scale_dev, self.x_trial)
            ctx.stencil_distance(self.x_trial, self.pool_t)
            ctx.energy_grad_scenes(self.x_trial, self.xt, self.pool_t, self.E_trial, self.g_trial)
            E2 = self.E_trial.cpu().numpy()
            Et = np.where(accepted, Et, E2)
            accepted = accepted | (E2 <= self.E_host)
        # every round recomputed the trial point of all scenes, the accepted
        # ones at their accepted scale, so x_trial and g_trial hold them
        keep = torch.as_tensor(accepted, device=self.x.device)[self.seg_dof]
        self.x = torch.where(keep, self.x_trial, self.x)
        self.g = torch.where(keep, self.g_trial, self.g)
        ctx.stencil_distance(self.x, self.pool)
        restart_next = np.array([o["restart_next"] for o in outs], bool)
        self.log.append(dict(k=self.k, restart=self.restart.copy(), accepted=accepted.copy(), scale=scale.copy(),
                             E=np.where(accepted, Et, self.E_host),
                             gnorm=np.sqrt([o["gnorm2"] for o in outs]),
                             mu=np.array([o["mu"] for o in outs]), nu=np.array([o["nu"] for o in outs])))
        self.E_host = np.where(accepted, Et, self.E_host)
        self.restart = (~accepted) | restart_next
        self.z, self.z_prev = self.z_prev, self.z
        self.k += 1
        return outs


class _PairBuffers:
    """Device outputs of one mas_constraint_set call (capacity cap)."""

    def __init__(self, cap, device, with_contacts=True):
        self.cap = cap
        self.pairs = torch.full((cap, 4), -1, dtype=torch.int32, device=device)
        self.kind = torch.zeros(cap, dtype=torch.uint8, device=device)
        self.dist = torch.zeros(cap, dtype=torch.float64, device=device)
        self.grad = torch.zeros(cap, 12, dtype=torch.float64, device=device) if with_contacts else None
        self.key = torch.zeros(cap, dtype=torch.int64, device=device) if with_contacts else None
        self.m = 0

    def contacts(self):
        m = self.m
        return DeviceContacts.from_tensors(self.key[:m], self.pairs[:m], self.grad[:m], self.dist[:m])


class GeoPNCG:
    """Algorithm 1 on the geometric point-triangle / edge-edge contacts of the
    scene's boundary surface, through the C ABI: ComputeConstraintSet at the
    head of each iteration (mas_constraint_set: distances, n = grad d and
    contact keys), RebuildMAS or the Woodbury update against it, z = P g,
    H_base z, the subspace step, ConservativeCCD for the per-subdomain steps
    (mas_ccd_safe_step over the pairs within ``radius``), and the descent
    check with the trial point's contact set (the energy's barrier is taken
    on the geometric distances).  The host reads per iteration the pair
    counts, the trial energy and the step scalars."""

    def __init__(self, scene, radius, block_prec="f64", levels=None, K=None, delta=0.3, hess_prec=None,
                 max_halvings=8, cap=None, device="cuda", deterministic=False):
        cfg = make_config(scene, levels=levels, K=K, block_prec=block_prec, hess_prec=hess_prec, delta=delta,
                          deterministic=deterministic)
        self.ctx = ctx = MasContext(scene, cfg, device=device)
        self.scene = scene
        self.radius = float(radius)
        self.max_halvings = max_halvings
        verts, tris, edges = synth.surface(scene.tets)
        r = ctx.rank
        self.vt = torch.as_tensor(r[verts].astype(np.int32), device=device)
        self.tt = torch.as_tensor(r[tris].astype(np.int32).reshape(-1, 3), device=device)
        self.et = torch.as_tensor(r[edges].astype(np.int32).reshape(-1, 2), device=device)
        max_contacts = cfg.max_contacts or max(2 * scene.X.shape[0], 65536)   # mas_create's default
        cap = cap or int(min(max_contacts, 8 * (len(verts) + len(edges)) + 4096))
        self.C = _PairBuffers(cap, device)          # contact set at x
        self.Ct = _PairBuffers(cap, device)         # contact set at the trial point
        self.cand = _PairBuffers(cap, device, with_contacts=False)
        v = ctx.vec
        self.x = ctx.to_lib(scene.x)
        self.xt = ctx.inertial_target(self.x, ctx.to_lib(scene.v))
        self.x_trial, self.g, self.g_trial = v(), v(), v()
        self.z, self.z_prev, self.vz, self.p, self.vp = v(), v(), v(), v(), v()
        self.E = torch.zeros(1, dtype=torch.float64, device=device)
        self.E_trial = torch.zeros(1, dtype=torch.float64, device=device)
        self.rank_hist = torch.zeros(max(cfg.max_rank, 0) + 1, dtype=torch.int32, device=device)
        self._set(self.x, self.C, self.scene.dhat)
        ctx.energy_grad(self.x, self.xt, self.C.contacts(), self.E, self.g)
        self.E_host = float(self.E.item())
        self.restart = True
        self.k = 0
        self.n_restarts = 0
        self.n_rejected = 0
        self.log = []

    def _set(self, x, buf, dist):
        with_c = buf.grad is not None
        n = self.ctx.constraint_set(x, self.vt, self.tt, self.et, dist, buf.pairs, buf.kind, buf.dist,
                                    buf.grad if with_c else None, buf.key if with_c else None)
        if n > buf.cap:
            raise RuntimeError("constraint set of %d pairs exceeds the capacity %d" % (n, buf.cap))
        buf.m = n
        return n

    def iterate(self):
        ctx = self.ctx
        C = self.C.contacts()
        if self.restart:
            ctx.build(self.x, C)
            self.n_restarts += 1
        else:
            ctx.woodbury_update(C, self.rank_hist)
        ctx.apply(self.g, self.z)
        ctx.hess_vec(self.z, with_update=False, y=self.vz)
        ctx.subspace_step(self.g, self.z, self.z_prev if self.k > 0 else None, self.vz, self.p, self.vp,
                          self.restart)
        st = ctx.step_out()
        if not (np.isfinite(st["mu"]) and np.isfinite(st["nu"])):
            # a block or capacitance factor failed: report the library's first error
            code, msg = ctx.sync()
            raise RuntimeError("GeoPNCG iteration %d: non-finite step scalars; library status %d (%s)"
                               % (self.k, code, msg))
        mc = self._set(self.x, self.cand, self.radius)
        ctx.ccd_safe_step(self.x, self.p, self.radius, self.cand.pairs, self.cand.kind, self.cand.dist, mc, 1.0,
                          self.x_trial)
        scale = 1.0
        accepted = False
        Et = float("inf")
        for h in range(self.max_halvings + 1):
            self._set(self.x_trial, self.Ct, self.scene.dhat)
            ctx.energy_grad(self.x_trial, self.xt, self.Ct.contacts(), self.E_trial, self.g_trial)
            Et = float(self.E_trial.item())
            if Et <= self.E_host:
                accepted = True
                break
            if h < self.max_halvings:
                scale *= 0.5
                ctx.safe_step(self.x, self.p, None, scale, self.x_trial)
        self.log.append(dict(k=self.k, gnorm=float(np.sqrt(st["gnorm2"])), mu=st["mu"], nu=st["nu"], r=st["r"],
                             restart=bool(self.restart), fallback=bool(st["fallback"]), E=self.E_host,
                             m=self.C.m, candidates=mc, scale=scale, accepted=accepted))
        if accepted:
            self.x, self.x_trial = self.x_trial, self.x
            self.g, self.g_trial = self.g_trial, self.g
            self.C, self.Ct = self.Ct, self.C
            self.E_host = Et
            self.restart = bool(st["restart_next"])
        else:
            self.n_rejected += 1
            self.restart = True
        self.z, self.z_prev = self.z_prev, self.z
        self.k += 1
        return st
