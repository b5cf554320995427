"""The PNCG loop of Algorithm 1 (FP64): on the affine contact pool
(``OraclePNCG``) and on geometric point-triangle / edge-edge contacts of a
boundary surface (``OracleGeoPNCG``).

Test infrastructure (see the package docstring).  Every iteration follows
Algorithm 1 with full-rebuild semantics for the preconditioner blocks:

1. constraint set: pool stencils with 0 < d(x_k) < dhat;
2. restart: assemble H_base at x_k with that set and rebuild every MAS
   level; otherwise classify against the base set, select Top-K per
   subdomain and invert the updated fine blocks directly;
3. g = grad E(x_k), z = P g, and the subspace step with H~ = H_base + U U^T;
4. per-subdomain safe steps, then the descent check: all step sizes are
   halved (at most 8 times) until E does not increase; if none does, x is
   kept and the next iteration restarts (the paper's line search is not
   described; this is the reading used here);
5. r_k = |g^T z_prev| / (g^T z) decides the next restart (threshold delta).
"""
from __future__ import annotations

import numpy as np

from . import constraint_set as CS
from . import contact, fem, jacobi, mas, woodbury, pncg


def pool_distance(pool, x):
    """d(x) = grad . x[idx] - off for the affine stencils."""
    return (pool['grad'] * fem.stencil_gather(pool['idx'], x)).sum(1) - pool['off']


RULES = {"fr": pncg.BETA_FR, "cd": pncg.BETA_CD, "dk": pncg.BETA_DK}


class OraclePNCG:
    """``update`` picks the preconditioner strategy of the ablation study
    (Section 5, preconditioner update strategy): "woodbury" (the method),
    "freeze" (the restart's MAS kept until the next restart: no Top-K
    columns, while H~ keeps the untruncated U) or "rebuild" (RebuildMAS at
    every iteration, the CG restart form still decided by the ratio test).
    ``rule`` picks the direction: "subspace" (the method's 2x2 step) or a
    comparison rule "fr", "cd", "dk" (``pncg.beta_step``).  ``precond``
    "bj3" replaces MAS by the 3x3 block-Jacobi inverse of H~ (the
    comparison preconditioner, ``oracle.jacobi``); ``hierarchy``
    "connectivity" groups the MAS levels by the connectivity-aware order
    (``mas.connectivity_perm``) instead of the Morton order."""

    def __init__(self, scene, levels=None, K=None, delta=0.3,
                 cos_rot=np.cos(np.deg2rad(25.0)), max_halvings=8, update="woodbury", rule="subspace",
                 precond="mas", hierarchy="morton"):
        if update not in ("woodbury", "freeze", "rebuild") or (rule != "subspace" and rule not in RULES) \
                or precond not in ("mas", "bj3"):
            raise ValueError("unknown update strategy, direction rule or preconditioner")
        self.update = update
        self.rule = rule
        self.precond = precond
        self.scene = scene
        self.prob = fem.Problem(scene)
        links = None
        if hierarchy == "connectivity":
            # every vertex pair of the pool stencils active at the start
            d = pool_distance(scene.pool, np.asarray(scene.x, np.float64).reshape(-1))
            idx = scene.pool['idx'][(d > 0) & (d < scene.dhat)]
            links = [(int(s[a]), int(s[b])) for s in idx for a in range(4) for b in range(a + 1, 4)
                     if s[a] >= 0 and s[b] >= 0]
            links = np.array(links, np.int64).reshape(-1, 2)
        self.hier = mas.Hierarchy(scene.X, levels or scene.levels, tets=scene.tets, order=hierarchy, links=links)
        self.K = 0 if update == "freeze" else (K or scene.K)
        self.g_prev = None
        self.d = None
        self.delta = delta
        self.cos_rot = cos_rot
        self.max_halvings = max_halvings
        self.pool = scene.pool
        self.x_tilde = fem.inertial_target(scene.x, scene.v, scene.h, scene.gravity).reshape(-1)
        self.x = np.asarray(scene.x, np.float64).reshape(-1).copy()
        self.restart = True
        self.p = np.zeros_like(self.x)
        self.z_prev = None
        self.log = []

    def constraint_set(self, x):
        d = pool_distance(self.pool, x)
        act = (d > 0) & (d < self.prob.dhat)
        return {'key': self.pool['key'][act], 'idx': self.pool['idx'][act],
                'grad': self.pool['grad'][act], 'd': d[act]}

    def iterate(self):
        prob, hier = self.prob, self.hier
        x = self.x
        C = self.constraint_set(x)
        bj = self.precond == "bj3"
        if self.restart or self.update == "rebuild":
            self.H_base = prob.assemble(x, C)
            if not bj:
                self.mas = mas.MAS(hier, self.H_base)
                blocks = self.mas.fine
            self.base = C
            U = None
        else:
            dS, u, _ = woodbury.classify(prob, self.base, C, self.cos_rot)
            if not bj:
                sel = woodbury.topk(hier, C, dS, u, self.K)
                blocks = woodbury.updated_blocks(hier, self.H_base, C, u, sel)
            U = woodbury.global_U(prob, C, u, dS)
        g = prob.gradient(x, self.x_tilde, C)
        if bj:
            Ht = self.H_base if U is None else self.H_base + U @ U.T
            z = jacobi.apply(jacobi.inverse_blocks(Ht), g)
        else:
            z = self.mas.apply(g, blocks)

        def Hmul(v):
            y = self.H_base @ v
            if U is not None:
                y = y + U @ (U.T @ v)
            return y

        if self.rule == "subspace":
            mu, nu, p, fb, *_ = pncg.subspace_step(g, z, self.p, Hmul, self.restart)
            d = p
        else:
            # mu, nu of the log hold alpha and beta
            mu, nu, d, p, fb = pncg.beta_step(RULES[self.rule], g, self.g_prev, z, self.z_prev, self.d, Hmul,
                                              self.restart)
        dpool = pool_distance(self.pool, x)
        alpha = pncg.safe_alpha(hier, self.pool['idx'], self.pool['grad'], dpool, p)
        E0 = prob.energy(x, self.x_tilde, C)
        accepted = False
        for _ in range(self.max_halvings + 1):
            xn = pncg.step_positions(hier, x, p, alpha)
            if prob.energy(xn, self.x_tilde, self.constraint_set(xn)) <= E0:
                accepted = True
                break
            alpha = 0.5 * alpha
        r = pncg.restart_ratio(g, self.z_prev, z) if self.z_prev is not None else 0.0
        self.log.append(dict(gnorm=float(np.linalg.norm(g)), znorm=float(np.linalg.norm(z)),
                             mu=mu, nu=nu, r=r, restart=self.restart, fallback=fb, E=E0,
                             m=int(C['key'].size), accepted=accepted))
        # without a decrease the point is kept and the next iteration restarts
        self.restart = (r > self.delta) or not accepted
        self.z_prev = z
        self.g_prev = g
        self.p = p
        self.d = d
        if accepted:
            self.x = xn
        return g, z, p


def pair_keys(pairs, kinds, verts, tris, edges):
    """Contact identities of geometric pairs (the reading of Section 4.1.1's
    contact identity): the kind (tag 2 point-triangle, 3 edge-edge, bits
    60-63) and the two primitives' indices in the surface lists, 30 bits
    each (vertex index in verts and triangle index in tris; the two edge
    indices, smaller first)."""
    vpos = {int(v): i for i, v in enumerate(verts)}
    tpos = {tuple(int(a) for a in t): i for i, t in enumerate(np.asarray(tris).reshape(-1, 3))}
    epos = {tuple(int(a) for a in e): i for i, e in enumerate(np.asarray(edges).reshape(-1, 2))}
    keys = np.zeros(len(pairs), np.uint64)
    for n, (p, k) in enumerate(zip(pairs, kinds)):
        if k == contact.PT:
            a, b = vpos[int(p[0])], tpos[tuple(int(q) for q in p[1:])]
        else:
            a, b = epos[(int(p[0]), int(p[1]))], epos[(int(p[2]), int(p[3]))]
            a, b = min(a, b), max(a, b)
        keys[n] = (np.uint64(2 + int(k)) << np.uint64(60)) | (np.uint64(a) << np.uint64(30)) | np.uint64(b)
    return keys


class OracleGeoPNCG:
    """Algorithm 1 on the geometric contacts of a boundary surface (verts,
    tris, edges): ComputeConstraintSet at the head of each iteration
    (brute force, ``oracle.constraint_set``) with distances and gradients
    from ``oracle.contact``; RebuildMAS or the Woodbury update against it;
    the subspace step; ConservativeCCD over the pairs within ``radius`` for
    the per-subdomain steps (``pncg.ccd_safe_alpha``); the descent check
    with the contact set of the trial point; the restart test."""

    def __init__(self, scene, surface, radius, levels=None, K=None, delta=0.3,
                 cos_rot=np.cos(np.deg2rad(25.0)), max_halvings=8):
        self.scene = scene
        self.verts, self.tris, self.edges = surface
        self.radius = float(radius)
        self.prob = fem.Problem(scene)
        self.hier = mas.Hierarchy(scene.X, levels or scene.levels)
        self.K = K or scene.K
        self.delta = delta
        self.cos_rot = cos_rot
        self.max_halvings = max_halvings
        self.x_tilde = fem.inertial_target(scene.x, scene.v, scene.h, scene.gravity).reshape(-1)
        self.x = np.asarray(scene.x, np.float64).reshape(-1).copy()
        self.restart = True
        self.p = np.zeros_like(self.x)
        self.z_prev = None
        self.log = []

    def pairs_within(self, x, dist):
        pairs, kinds, d = CS.constraint_set(x, self.verts, self.tris, self.edges, dist)
        return np.asarray(pairs, np.int64).reshape(-1, 4), np.asarray(kinds, np.int64), np.asarray(d)

    def constraint_set(self, x):
        pairs, kinds, _ = self.pairs_within(x, self.prob.dhat)
        d, grad, _ = contact.contact_distances(x, pairs, kinds)
        return {'key': pair_keys(pairs, kinds, self.verts, self.tris, self.edges), 'idx': pairs,
                'grad': grad, 'd': d, 'kind': kinds}

    def iterate(self):
        prob, hier = self.prob, self.hier
        x = self.x
        C = self.constraint_set(x)
        if self.restart:
            self.H_base = prob.assemble(x, C)
            self.mas = mas.MAS(hier, self.H_base)
            self.base = C
            blocks = self.mas.fine
            U = None
        else:
            dS, u, _ = woodbury.classify(prob, self.base, C, self.cos_rot)
            sel = woodbury.topk(hier, C, dS, u, self.K)
            blocks = woodbury.updated_blocks(hier, self.H_base, C, u, sel)
            U = woodbury.global_U(prob, C, u, dS)
        g = prob.gradient(x, self.x_tilde, C)
        z = self.mas.apply(g, blocks)

        def Hmul(v):
            y = self.H_base @ v
            if U is not None:
                y = y + U @ (U.T @ v)
            return y

        mu, nu, p, fb, *_ = pncg.subspace_step(g, z, self.p, Hmul, self.restart)
        cp, ck, cd = self.pairs_within(x, self.radius)
        alpha = pncg.ccd_safe_alpha(hier, x, p, self.radius, cp, ck, cd)
        E0 = prob.energy(x, self.x_tilde, C)
        accepted = False
        scale = 1.0
        for _ in range(self.max_halvings + 1):
            xn = pncg.step_positions(hier, x, p, scale * alpha)
            if prob.energy(xn, self.x_tilde, self.constraint_set(xn)) <= E0:
                accepted = True
                break
            scale *= 0.5
        r = pncg.restart_ratio(g, self.z_prev, z) if self.z_prev is not None else 0.0
        self.log.append(dict(gnorm=float(np.linalg.norm(g)), znorm=float(np.linalg.norm(z)),
                             mu=mu, nu=nu, r=r, restart=self.restart, fallback=fb, E=E0,
                             m=int(C['key'].size), accepted=accepted, alpha=alpha, scale=scale,
                             candidates=int(len(cp))))
        self.restart = (r > self.delta) or not accepted
        self.z_prev = z
        self.p = p
        if accepted:
            self.x = xn
        return g, z, p
