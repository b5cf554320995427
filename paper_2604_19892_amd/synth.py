"""Seeded synthetic scenes shaped like the paper's workloads.

This module only produces *inputs*: rest and current vertex positions,
tetrahedra, material constants, time-step constants and contact stencils.
It holds none of the solver's arithmetic (no element quantities, no
barrier, no preconditioner); the library and the oracle each derive
everything else from these arrays on their own.

Contact model.  A contact is an affine distance stencil over at most four
vertices: ``d(x) = sum_j grad[j] . x[idx[j]] - off`` (``idx`` padded with
-1, ``grad`` the 12-vector dd/dx of the stencil).  Point-plane contacts
(one vertex), point-triangle and edge-edge stencils (four vertices, weights
from barycentric / edge parameters) all take this form.  The paper's
scenes use real primitive pairs (Section 4.1 and Table 1); these affine
stand-ins keep the contact Hessian exactly rank one, which is the structure
the Woodbury update (Section 4.1) relies on.

Scenes (sizes follow the paper's workloads, Table 1):
  * ``grid_scene``       8x8x8 lattice, point-plane contacts (small case)
  * ``two_boxes_scene``  two stacked 40x40x20 boxes, PT/EE stencils
  * ``stacked_boxes_scene`` two boxes a fraction of dhat apart, one falling
                         onto the other (geometric contacts of the surface)
  * ``puffer_scene``     eight spiky balls, ~1.14M vertices / ~2.72M tets,
                         ~1M active contacts (the Puffer Balls shape)
"""
from __future__ import annotations

import dataclasses
import numpy as np

# contact type tags stored in the top bits of the key
KEY_PLANE = 1
KEY_PT = 2
KEY_EE = 3


@dataclasses.dataclass
class Scene:
    name: str
    X: np.ndarray          # (N,3) rest positions
    x: np.ndarray          # (N,3) positions at the start of the step
    v: np.ndarray          # (N,3) velocities at the start of the step
    tets: np.ndarray       # (T,4) int32 vertex ids (positive orientation)
    density: np.ndarray    # (T,)
    youngs: np.ndarray     # (T,)
    poisson: np.ndarray    # (T,)
    h: float               # time step
    dhat: float            # barrier activation distance
    kappa: float           # barrier stiffness scale
    gravity: np.ndarray    # (3,) acceleration
    pool: dict             # affine contact candidates: key,idx,grad,off
    levels: int            # MAS levels (level 0 + coarse levels)
    K: int                 # Top-K per subdomain

    @property
    def N(self):
        return self.X.shape[0]

    @property
    def T(self):
        return self.tets.shape[0]


# ---------------------------------------------------------------- lattices

def lattice_from_cubes(cubes, edge, origin):
    """Mesh made of unit cubes at integer lattice coordinates ``cubes``
    (M,3).  Returns (X, tets).  Cubes with odd coordinate sum use the
    mirrored five-tet split, so the face diagonals of neighbours agree."""
    cubes = np.asarray(cubes, dtype=np.int64)
    offs = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)],
                    dtype=np.int64)  # corner order: index = a + 2b + 4c
    corners = cubes[:, None, :] + offs[None, :, :]            # (M,8,3)
    lo = corners.reshape(-1, 3).min(0)
    span = corners.reshape(-1, 3).max(0) - lo + 1
    code = ((corners[..., 0] - lo[0]) * span[1] + (corners[..., 1] - lo[1])) * span[2] \
        + (corners[..., 2] - lo[2])
    uniq, inv = np.unique(code.reshape(-1), return_inverse=True)
    vid = inv.reshape(-1, 8).astype(np.int64)
    c2 = uniq % span[2] + lo[2]
    r = uniq // span[2]
    c1 = r % span[1] + lo[1]
    c0 = r // span[1] + lo[0]
    X = np.stack([c0, c1, c2], 1).astype(np.float64) * edge + np.asarray(origin, np.float64)

    def C(a, b, c):
        return a + 2 * b + 4 * c

    even = [
        (C(0, 0, 0), C(1, 0, 0), C(0, 1, 0), C(0, 0, 1)),
        (C(1, 1, 0), C(1, 0, 0), C(0, 1, 0), C(1, 1, 1)),
        (C(1, 0, 1), C(1, 0, 0), C(0, 0, 1), C(1, 1, 1)),
        (C(0, 1, 1), C(0, 1, 0), C(0, 0, 1), C(1, 1, 1)),
        (C(1, 0, 0), C(0, 1, 0), C(0, 0, 1), C(1, 1, 1)),
    ]

    def mirror(k):  # a -> 1-a
        a, b, c = k & 1, (k >> 1) & 1, (k >> 2) & 1
        return C(1 - a, b, c)

    odd = [tuple(mirror(k) for k in t) for t in even]
    parity = (cubes.sum(1) & 1).astype(bool)
    te = vid[:, np.array(even)]                              # (M,5,4)
    to = vid[:, np.array(odd)]
    tets = np.where(parity[:, None, None], to, te).reshape(-1, 4)
    # positive orientation
    p = X[tets]
    det = np.einsum('ij,ij->i', np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    flip = det < 0
    tets[flip, 2], tets[flip, 3] = tets[flip, 3].copy(), tets[flip, 2].copy()
    return X, tets.astype(np.int32)


def box_cubes(nx, ny, nz):
    """Cube coordinates of an nx*ny*nz-vertex box."""
    g = np.stack(np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1),
                             indexing='ij'), -1)
    return g.reshape(-1, 3)


def _perturb(rng, X, tets, sigma, tries=20):
    """x = X + sigma*N(0,1), resampled until no tet is inverted."""
    for _ in range(tries):
        x = X + sigma * rng.standard_normal(X.shape)
        p = x[tets]
        det = np.einsum('ij,ij->i', np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]),
                        p[:, 3] - p[:, 0])
        if np.all(det > 0):
            return x
    raise RuntimeError("could not sample an uninverted displacement")


def _unit(rng, n):
    u = rng.standard_normal((n, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def _tilt(rng, base, max_deg):
    """Unit vectors within max_deg of the unit vectors ``base`` (n,3)."""
    n = base.shape[0]
    a = rng.standard_normal((n, 3))
    a -= (a * base).sum(1, keepdims=True) * base
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    ang = np.deg2rad(max_deg) * rng.uniform(0.0, 1.0, n)
    return np.cos(ang)[:, None] * base + np.sin(ang)[:, None] * a


def _make_key(tag, ids):
    """Identity key: type tag and sorted primitive ids (13 bits tag+hash)."""
    s = np.sort(ids, axis=1).astype(np.uint64)
    h = np.zeros(ids.shape[0], dtype=np.uint64)
    with np.errstate(over='ignore'):
        for j in range(s.shape[1]):
            h = h * np.uint64(1000003) + s[:, j] + np.uint64(1)
    return (np.uint64(tag) << np.uint64(60)) | (h & np.uint64((1 << 60) - 1))


def stencil_pool(key, idx, grad, x, d):
    """Affine pool entries with offsets chosen so that d(x) = d."""
    xs = np.where(idx[..., None] >= 0, x[np.maximum(idx, 0)], 0.0).reshape(-1, 12)
    off = (grad * xs).sum(1) - d
    return dict(key=np.ascontiguousarray(key, np.uint64),
                idx=np.ascontiguousarray(idx, np.int32),
                grad=np.ascontiguousarray(grad, np.float64),
                off=np.ascontiguousarray(off, np.float64))


def pool_distance(pool, x):
    """Distance of each affine stencil at positions x (definition of the
    synthetic contact model)."""
    idx = pool['idx']
    xs = np.where(idx[..., None] >= 0, x[np.maximum(idx, 0)], 0.0).reshape(-1, 12)
    return (pool['grad'] * xs).sum(1) - pool['off']


def contact_set(key, idx, grad, d):
    return dict(key=np.ascontiguousarray(key, np.uint64),
                idx=np.ascontiguousarray(idx, np.int32),
                grad=np.ascontiguousarray(grad, np.float64),
                d=np.ascontiguousarray(d, np.float64))


def subset(cs, sel):
    return {k: np.ascontiguousarray(v[sel]) for k, v in cs.items()}


def concat(*sets):
    return {k: np.ascontiguousarray(np.concatenate([s[k] for s in sets])) for k in sets[0]}


# -------------------------------------------------------- small grid scene

def grid_scene(n=8, seed=0, n_contacts=200, dhat=1e-3, h=0.01, E=1e5, nu=0.4, rho=1000.0,
               levels=2, K=8):
    """n^3-vertex unit cube, five tets per cube, random displacement of
    5% of the edge, ``n_contacts`` point-plane contacts with distances
    uniform in (1e-5, dhat)."""
    rng = np.random.default_rng(seed)
    edge = 1.0 / (n - 1)
    X, tets = lattice_from_cubes(box_cubes(n, n, n), edge, (0, 0, 0))
    x = _perturb(rng, X, tets, 0.05 * edge)
    T = tets.shape[0]
    pts = rng.choice(X.shape[0], n_contacts, replace=False)
    nrm = _unit(rng, n_contacts)
    d = rng.uniform(1e-5, dhat, n_contacts)
    idx = np.full((n_contacts, 4), -1, np.int32)
    idx[:, 0] = pts
    grad = np.zeros((n_contacts, 12))
    grad[:, :3] = nrm
    key = (np.uint64(KEY_PLANE) << np.uint64(60)) | np.arange(n_contacts, dtype=np.uint64)
    pool = stencil_pool(key, idx, grad, x, d)
    return Scene("grid%d" % n, X, x, np.zeros_like(X), tets,
                 np.full(T, rho), np.full(T, E), np.full(T, nu), h, dhat,
                 kappa=rho * edge ** 3, gravity=np.array([0.0, 0.0, -9.81]),
                 pool=pool, levels=levels, K=K)


def grid_update_sets(scene, seed=100):
    """Scripted base/current contact sets for the small grid scene.

    From the 200 base point-plane contacts: 50 are released, 50 stiffen
    (distance halved), 25 rotate (normal turned 40 degrees), 25 soften
    (distance times U(1.1,3), capped below dhat), 50 are unchanged, and 50
    new contacts appear.  Returns (C_base, C_curr) as contact sets with
    explicit distances."""
    rng = np.random.default_rng(seed)
    pool = scene.pool
    d0 = pool_distance(pool, scene.x)
    base = contact_set(pool['key'], pool['idx'], pool['grad'], d0)
    m = base['key'].shape[0]
    perm = rng.permutation(m)
    rel, stf, rot, sof, keep = np.split(perm, [50, 100, 125, 150])
    d_stf = base['d'][stf] * 0.5
    d_sof = np.minimum(base['d'][sof] * rng.uniform(1.1, 3.0, sof.size), 0.99 * scene.dhat)
    g_rot = base['grad'][rot].copy()
    n0 = g_rot[:, :3]
    a = rng.standard_normal((rot.size, 3))
    a -= (a * n0).sum(1, keepdims=True) * n0
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    th = np.deg2rad(40.0)
    g_rot[:, :3] = np.cos(th) * n0 + np.sin(th) * a
    cur_parts = [
        contact_set(base['key'][keep], base['idx'][keep], base['grad'][keep], base['d'][keep]),
        contact_set(base['key'][stf], base['idx'][stf], base['grad'][stf], d_stf),
        contact_set(base['key'][rot], base['idx'][rot], g_rot, base['d'][rot]),
        contact_set(base['key'][sof], base['idx'][sof], base['grad'][sof], d_sof),
    ]
    nn = 50
    pts = rng.choice(scene.N, nn, replace=False)
    idx = np.full((nn, 4), -1, np.int32)
    idx[:, 0] = pts
    grad = np.zeros((nn, 12))
    grad[:, :3] = _unit(rng, nn)
    key = (np.uint64(KEY_PLANE) << np.uint64(60)) | (np.arange(nn, dtype=np.uint64) + np.uint64(10000))
    cur_parts.append(contact_set(key, idx, grad, rng.uniform(1e-5, scene.dhat, nn)))
    cur = concat(*cur_parts)
    sh = rng.permutation(cur['key'].shape[0])
    return base, subset(cur, sh)


# ------------------------------------------------------ PT / EE stencils

def _pt_ee_stencils(rng, Xa, ids_a, quads_b, Xb_of, n_pt, n_ee, nrm_hint, tilt_deg, kq=6):
    """Point-triangle and edge-edge stencils between point set A (ids_a,
    positions Xa) and a quad surface B (quads_b (Q,4) vertex ids, quad
    centres Xb_of (Q,3)).  Each stencil pairs a random A vertex with one of
    its ``kq`` nearest B quads.  Returns idx (n,4), grad (n,12), tag (n,)."""
    from scipy.spatial import cKDTree
    tree = cKDTree(Xb_of)
    kq = min(kq, Xb_of.shape[0])

    def near(pts):
        _, q = tree.query(pts, k=kq)
        q = q.reshape(pts.shape[0], kq)
        return q[np.arange(pts.shape[0]), rng.integers(0, kq, pts.shape[0])]

    # point-triangle
    pa = rng.integers(0, ids_a.size, n_pt)
    qi = near(Xa[pa])
    tri_pick = rng.integers(0, 4, n_pt)               # which corner is dropped
    q = quads_b[qi]
    keep = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])[tri_pick]
    tri = np.take_along_axis(q, keep, 1)
    w = rng.dirichlet(np.ones(3), n_pt)
    n = _tilt(rng, np.repeat(nrm_hint[None], n_pt, 0), tilt_deg)
    idx_pt = np.concatenate([ids_a[pa][:, None], tri], 1)
    grad_pt = np.concatenate([n, -w[:, 0:1] * n, -w[:, 1:2] * n, -w[:, 2:3] * n], 1)
    # edge-edge: A edge = (vertex, another A vertex adjacent in id list)
    ea = rng.integers(0, ids_a.size - 1, n_ee)
    qj = near(Xa[ea])
    e_pick = rng.integers(0, 4, n_ee)
    qb = quads_b[qj]
    b0 = np.take_along_axis(qb, e_pick[:, None], 1)[:, 0]
    b1 = np.take_along_axis(qb, ((e_pick + 1) % 4)[:, None], 1)[:, 0]
    s = rng.uniform(0, 1, n_ee)
    t = rng.uniform(0, 1, n_ee)
    n2 = _tilt(rng, np.repeat(nrm_hint[None], n_ee, 0), tilt_deg)
    idx_ee = np.stack([ids_a[ea], ids_a[ea + 1], b0, b1], 1)
    grad_ee = np.concatenate([(1 - s)[:, None] * n2, s[:, None] * n2,
                              -(1 - t)[:, None] * n2, -t[:, None] * n2], 1)
    idx = np.concatenate([idx_pt, idx_ee]).astype(np.int32)
    grad = np.concatenate([grad_pt, grad_ee])
    tag = np.concatenate([np.full(n_pt, KEY_PT), np.full(n_ee, KEY_EE)])
    return idx, grad, tag


def _dedupe(idx, grad, tag):
    keys = np.concatenate([_make_key(KEY_PT, idx[tag == KEY_PT]),
                           _make_key(KEY_EE, idx[tag == KEY_EE])])
    order = np.concatenate([np.nonzero(tag == KEY_PT)[0], np.nonzero(tag == KEY_EE)[0]])
    idx, grad = idx[order], grad[order]
    # distinct vertices inside a stencil and unique keys
    s = np.sort(idx, 1)
    ok = np.all(s[:, 1:] != s[:, :-1], 1)
    _, first = np.unique(keys, return_index=True)
    sel = np.zeros(keys.size, bool)
    sel[first] = True
    sel &= ok
    return keys[sel], idx[sel], grad[sel]


def _loguniform(rng, lo, hi, n):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


# ---------------------------------------------------------- two boxes

def two_boxes_scene(seed=1, n_contacts=20000, dhat=1e-3, h=0.01, E=1e5, nu=0.4, rho=1000.0,
                    levels=3, K=8, nxy=40, nz=20, active_frac=1.0, kappa_scale=1.0, edge=None):
    """Two 40x40x20-vertex boxes (edge 1/39: unit boxes, unless ``edge`` is
    given) stacked with the upper box offset by half an edge in x and y; PT
    and EE stencils between the facing layers with distances log-uniform in
    (1e-6, dhat) and normals within 10 degrees of the vertical.  Barrier
    stiffness kappa_scale * rho * edge^3."""
    rng = np.random.default_rng(seed)
    edge = 1.0 / (nxy - 1) if edge is None else float(edge)
    Xl, tl = lattice_from_cubes(box_cubes(nxy, nxy, nz), edge, (0, 0, 0))
    z0 = (nz - 1) * edge + 0.5 * dhat
    Xu, tu = lattice_from_cubes(box_cubes(nxy, nxy, nz), edge, (0.5 * edge, 0.5 * edge, z0))
    X = np.concatenate([Xl, Xu])
    tets = np.concatenate([tl, tu + Xl.shape[0]]).astype(np.int32)
    x = _perturb(rng, X, tets, 0.01 * edge)
    nl = Xl.shape[0]
    top_l = np.nonzero(np.isclose(Xl[:, 2], (nz - 1) * edge))[0]
    bot_u = np.nonzero(np.isclose(Xu[:, 2], z0))[0] + nl

    def quads(ids, Xs):
        # quads of a planar lattice layer given its vertex ids (sorted by x,y)
        ij = np.round((Xs[ids][:, :2] - Xs[ids][:, :2].min(0)) / edge).astype(np.int64)
        lut = -np.ones((nxy, nxy), np.int64)
        lut[ij[:, 0], ij[:, 1]] = ids
        a = lut[:-1, :-1].ravel()
        b = lut[1:, :-1].ravel()
        c = lut[1:, 1:].ravel()
        d = lut[:-1, 1:].ravel()
        qd = np.stack([a, b, c, d], 1)
        cen = 0.25 * (Xs[a] + Xs[b] + Xs[c] + Xs[d])
        return qd, cen

    ql, cl = quads(top_l, X)
    qu, cu = quads(bot_u, X)
    n_pool = int(round(n_contacts / active_frac))
    half = int(n_pool * 0.75)        # oversample; duplicates are dropped
    i1, g1, t1 = _pt_ee_stencils(rng, X[bot_u], bot_u, ql, cl, int(half * 0.7), half - int(half * 0.7),
                                 np.array([0, 0, 1.0]), 10.0)
    i2, g2, t2 = _pt_ee_stencils(rng, X[top_l], top_l, qu, cu, int(half * 0.7), half - int(half * 0.7),
                                 np.array([0, 0, -1.0]), 10.0)
    key, idx, grad = _dedupe(np.concatenate([i1, i2]), np.concatenate([g1, g2]),
                             np.concatenate([t1, t2]))
    sel = rng.permutation(key.size)[:n_pool]
    key, idx, grad = key[sel], idx[sel], grad[sel]
    m = key.size
    n_act = int(round(m * active_frac))
    d = np.concatenate([_loguniform(rng, 1e-6, dhat, n_act),
                        rng.uniform(1.05 * dhat, 3 * dhat, m - n_act)])
    rng.shuffle(d)
    pool = stencil_pool(key, idx, grad, x, d)
    T = tets.shape[0]
    return Scene("two_boxes", X, x, np.zeros_like(X), tets,
                 np.full(T, rho), np.full(T, E), np.full(T, nu), h, dhat,
                 kappa=kappa_scale * rho * edge ** 3, gravity=np.array([0.0, 0.0, -9.81]),
                 pool=pool, levels=levels, K=K)


def stacked_boxes_scene(seed=4, nxy=10, nz=5, dhat=1e-3, h=0.01, E=1e5, nu=0.4, rho=1000.0, levels=2, K=8,
                        gap=0.5, speed=0.5, kappa_scale=1e3):
    """Two boxes for geometric contacts: the upper one (offset by half an
    edge in x and y) rests gap * dhat above the lower one and moves down at
    ``speed`` (its inertial target lies far inside the lower box, so the
    barrier has to hold it); vertex noise of 0.05 gap * dhat keeps the start
    free of intersections.  No contact pool: the contacts are the boundary
    surface's point-triangle and edge-edge pairs within dhat.

    The barrier stiffness is kappa_scale * rho * edge^3, as for the puffer
    balls: at kappa_scale = 1 the CCD-limited steps let surface pairs close
    to 1e-12 and below (the safe step only keeps them apart), where the
    barrier's curvature puts the blocks beyond float64 Cholesky."""
    rng = np.random.default_rng(seed)
    edge = 1.0 / (nxy - 1)
    Xl, tl = lattice_from_cubes(box_cubes(nxy, nxy, nz), edge, (0, 0, 0))
    z0 = (nz - 1) * edge + gap * dhat
    Xu, tu = lattice_from_cubes(box_cubes(nxy, nxy, nz), edge, (0.5 * edge, 0.5 * edge, z0))
    X = np.concatenate([Xl, Xu])
    tets = np.concatenate([tl, tu + Xl.shape[0]]).astype(np.int32)
    x = _perturb(rng, X, tets, 0.05 * gap * dhat)
    v = np.zeros_like(X)
    v[Xl.shape[0]:, 2] = -speed
    T = tets.shape[0]
    empty = stencil_pool(np.zeros(0, np.uint64), np.zeros((0, 4), np.int32), np.zeros((0, 12)), x, np.zeros(0))
    return Scene("stacked_boxes", X, x, v, tets, np.full(T, rho), np.full(T, E), np.full(T, nu), h, dhat,
                 kappa=kappa_scale * rho * edge ** 3, gravity=np.array([0.0, 0.0, -9.81]), pool=empty,
                 levels=levels, K=K)


def combs_scene(seed=3, teeth=8, width=2, tooth_len=12, base=2, depth=4, dhat=1e-3, h=0.01, E=1e5, nu=0.4,
                rho=1000.0, levels=2, K=8, kappa_scale=1.0):
    """Two combs whose teeth interleave one lattice edge apart (edge 1/32):
    parts that are close in space but not connected, the case where a
    Morton grouping puts vertices of both combs into one subdomain.  Teeth
    ``width`` cubes wide, ``tooth_len`` long and ``depth`` deep hang from
    slabs ``base`` cubes thick.  Affine point-point stencils join facing
    vertices of neighbouring teeth (d = x_B - x_A along the x axis minus an
    offset), with distances log-uniform in (1e-6, dhat).  Barrier stiffness
    kappa_scale * rho * edge^3 (the blocks' condition numbers stay near 1e6
    at the default, as on the grid and two-box scenes)."""
    rng = np.random.default_rng(seed)
    edge = 1.0 / 32
    pitch = width + 1
    nxc = 2 * teeth * pitch
    ca, cb = [], []
    for i in range(nxc):
        for k in range(depth):
            for j in range(base):
                ca.append((i, j, k))
                cb.append((i, base + 1 + tooth_len + j, k))
    for t in range(teeth):
        for i in range(width):
            for j in range(tooth_len):
                for k in range(depth):
                    ca.append((2 * t * pitch + i, base + j, k))
                    cb.append(((2 * t + 1) * pitch + i, base + 1 + j, k))
    XA, tA = lattice_from_cubes(np.array(ca), edge, (0.0, 0.0, 0.0))
    XB, tB = lattice_from_cubes(np.array(cb), edge, (0.0, 0.0, 0.0))
    X = np.concatenate([XA, XB])
    tets = np.concatenate([tA, tB + XA.shape[0]]).astype(np.int32)
    x = _perturb(rng, X, tets, 0.01 * edge)
    # facing tooth faces: A tooth t's right face and B tooth t's left face
    lut = {tuple(np.round(p / edge).astype(np.int64)): i for i, p in enumerate(XB)}
    pairs = []
    for t in range(teeth):
        xa = 2 * t * pitch + width
        for ia in np.nonzero(np.round(XA[:, 0] / edge).astype(np.int64) == xa)[0]:
            q = np.round(XA[ia] / edge).astype(np.int64)
            if q[1] < base + 1:
                continue
            jb = lut.get((xa + 1, int(q[1]), int(q[2])))
            if jb is not None:
                pairs.append((ia, jb + XA.shape[0]))
    pairs = np.array(pairs, np.int64)
    m = pairs.shape[0]
    idx = -np.ones((m, 4), np.int32)
    idx[:, :2] = pairs
    grad = np.zeros((m, 12))
    grad[:, 0] = -1.0
    grad[:, 3] = 1.0
    d = _loguniform(rng, 1e-6, dhat, m)
    key = _make_key(KEY_PT, pairs)
    pool = stencil_pool(key, idx, grad, x, d)
    T = tets.shape[0]
    return Scene("combs", X, x, np.zeros_like(X), tets, np.full(T, rho), np.full(T, E), np.full(T, nu), h, dhat,
                 kappa=kappa_scale * rho * edge ** 3, gravity=np.array([0.0, 0.0, -9.81]), pool=pool,
                 levels=levels, K=K)


def batch_scene(n_scenes=64, seed=11, size_range=(5e3, 1.2e5), contact_range=(1e3, 4e4), levels=3, K=24,
                dhat=1e-3, h=0.01, rho=1000.0, kappa=1e3 * 1000.0 / 39 ** 3, speed=0.5, spacing=2.0):
    """Independent scenes in one mesh: each a pair of stacked boxes (two_boxes
    layout, lattice edge 1/39 in every scene, so the boxes grow with the
    vertex count and one kappa suits all) with a vertex count log-uniform in
    ``size_range`` and a stencil count log-uniform in ``contact_range``
    (capped by what its facing layers hold), the upper box moving down at
    ``speed``; scenes sit ``spacing`` apart on a 4-wide grid, so they share
    no tet and no stencil.  Returns the combined scene and the vertex offset
    of each scene (n_scenes + 1)."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(size_range[0]), np.log(size_range[1]), n_scenes))
    counts = np.exp(rng.uniform(np.log(contact_range[0]), np.log(contact_range[1]), n_scenes))
    Xs, xs, vs, ts, pools, offs = [], [], [], [], [], [0]
    for i in range(n_scenes):
        nxy = max(8, int(round(sizes[i] ** (1.0 / 3.0))))
        nz = max(4, nxy // 2)
        cap = 8 * nxy * nxy
        sc = two_boxes_scene(seed=seed * 1000 + i, n_contacts=int(min(counts[i], cap)), dhat=dhat, h=h, rho=rho,
                             levels=levels, K=K, nxy=nxy, nz=nz, active_frac=0.8, edge=1.0 / 39)
        shift = spacing * np.array([i % 4, (i // 4) % 4, i // 16], np.float64)
        o = offs[-1]
        Xs.append(sc.X + shift)
        xs.append(sc.x + shift)
        v = np.zeros_like(sc.X)
        v[sc.N // 2:, 2] = -speed
        vs.append(v)
        ts.append(sc.tets + o)
        idx = np.where(sc.pool['idx'] >= 0, sc.pool['idx'] + o, -1).astype(np.int32)
        tag = sc.pool['key'] >> np.uint64(60)
        key = (tag << np.uint64(60)) | (np.uint64(i) << np.uint64(52)) | (sc.pool['key'] & np.uint64((1 << 52) - 1))
        pools.append(dict(key=key, idx=idx, grad=sc.pool['grad'], off=sc.pool['off'] + (sc.pool['grad'].reshape(
            -1, 4, 3) * np.where(sc.pool['idx'][..., None] >= 0, shift, 0.0)).sum((1, 2))))
        offs.append(o + sc.N)
    X = np.concatenate(Xs)
    tets = np.concatenate(ts).astype(np.int32)
    pool = {k: np.concatenate([p[k] for p in pools]) for k in ("key", "idx", "grad", "off")}
    T = tets.shape[0]
    out = Scene("batch%d" % n_scenes, X, np.concatenate(xs), np.concatenate(vs), tets, np.full(T, rho),
                np.full(T, 1e5), np.full(T, 0.4), h, dhat, kappa=kappa, gravity=np.array([0.0, 0.0, -9.81]),
                pool=pool, levels=levels, K=K)
    return out, np.array(offs, np.int64)


def churn_set(rng, scene, base, frac=0.3):
    """Scripted contact churn of a fraction ``frac`` of a contact set:
    40% replaced by fresh stencils (new keys), 30% stiffen (distance x
    U(0.1,0.9)), 15% rotate (normal turned 30-90 degrees), 15% soften
    (distance x U(1.1,3) capped below dhat).  Returns the current set."""
    m = base['key'].shape[0]
    nch = int(round(frac * m))
    perm = rng.permutation(m)
    ch = perm[:nch]
    keep = perm[nch:]
    n_rep = int(0.4 * nch)
    n_stf = int(0.3 * nch)
    n_rot = int(0.15 * nch)
    rep, stf, rot, sof = np.split(ch, [n_rep, n_rep + n_stf, n_rep + n_stf + n_rot])
    parts = [subset(base, keep)]
    s = subset(base, stf)
    s['d'] = s['d'] * rng.uniform(0.1, 0.9, stf.size)
    parts.append(s)
    r = subset(base, rot)
    g = r['grad'].reshape(-1, 4, 3)
    nz = np.linalg.norm(g, axis=2)
    j = np.argmax(nz, 1)
    n0 = g[np.arange(g.shape[0]), j] / nz[np.arange(g.shape[0]), j][:, None]
    a = rng.standard_normal(n0.shape)
    a -= (a * n0).sum(1, keepdims=True) * n0
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    th = np.deg2rad(rng.uniform(30, 90, n0.shape[0]))
    n1 = np.cos(th)[:, None] * n0 + np.sin(th)[:, None] * a
    # rotate every stencil block with the same rotation taking n0 to n1
    w = nz / nz[np.arange(g.shape[0]), j][:, None]
    sign = np.sign((g * n0[:, None, :]).sum(2))
    r['grad'] = (sign[..., None] * w[..., None] * n1[:, None, :]).reshape(-1, 12)
    parts.append(r)
    so = subset(base, sof)
    so['d'] = np.minimum(so['d'] * rng.uniform(1.1, 3.0, sof.size), 0.99 * scene.dhat)
    parts.append(so)
    # replacements: reuse the stencils' vertex sets of other pool members with fresh keys
    src = rng.integers(0, m, rep.size)
    nw = subset(base, src)
    nw['key'] = (np.uint64(7) << np.uint64(60)) | (rng.integers(0, 1 << 40, rep.size).astype(np.uint64))
    nw['d'] = _loguniform(rng, 1e-6, scene.dhat, rep.size)
    parts.append(nw)
    cur = concat(*parts)
    _, first = np.unique(cur['key'], return_index=True)
    cur = subset(cur, np.sort(first))
    return subset(cur, rng.permutation(cur['key'].shape[0]))


# ---------------------------------------------------------- puffer balls

def puffer_scene(seed=2, n_balls_axis=2, core=(36, 36, 37), n_spikes=1182, spike_len=20,
                 pool_size=1_250_000, active_frac=0.8, dhat=1e-4, h=0.005, E=1e5, nu=0.4,
                 rho=1000.0, ball_size=0.2, levels=4, K=8, speed=0.5, kappa_scale=1e3, dmin=1e-7):
    """Eight spiky balls in a 2x2x2 arrangement.  Each ball is a lattice
    core plus radial 2x2-vertex spike columns standing on its faces; the
    spikes of face-adjacent balls interleave, and the contact stencils
    (PT and EE) are drawn between those interleaved spikes.  With the
    defaults: 1,140,096 vertices, 2,709,600 tets, 1.25M candidate stencils
    of which 80% start active (distance log-uniform in (dmin, dhat)).
    Velocities point toward the scene centre at ``speed``.

    The barrier stiffness is kappa_scale * rho * edge^3 (the paper leaves
    kappa open).  With kappa_scale = 1e3 (kappa ~ 0.17) the barrier force of
    a stencil balances the inertial push of a vertex (mass rho edge^3 moved
    h * speed toward the centre) at a distance of about 1e-7, inside the
    initial distance range; at kappa_scale = 1 that balance sits near
    1e-10, stencils pushed by several vertices close to 1e-14 and below,
    and the descent check then rejects every trial point (the barrier's
    curvature changes by orders of magnitude within one step)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = core
    edge = ball_size / (max(core) - 1)
    core_cubes = box_cubes(nx, ny, nz)
    hi = np.array([nx - 1, ny - 1, nz - 1])
    # candidate spike sites: stride-2 quads on each face
    sites = []
    for ax in range(3):
        o1, o2 = [a for a in range(3) if a != ax]
        u = np.arange(0, hi[o1], 2)
        w = np.arange(0, hi[o2], 2)
        U, W = np.meshgrid(u, w, indexing='ij')
        for side in (0, 1):
            s = np.zeros((U.size, 5), np.int64)
            s[:, 0] = ax
            s[:, 1] = side
            s[:, 2] = U.ravel()
            s[:, 3] = W.ravel()
            sites.append(s)
    sites = np.concatenate(sites)
    Xs, tets_l, ball_of_v, face_v = [], [], [], []
    nv = 0
    centre_grid = (n_balls_axis - 1) / 2.0
    pitch = (hi + spike_len) * edge + 0.37 * edge      # facing spikes interleave fully
    ball_ids = []
    for bi in range(n_balls_axis ** 3):
        b = np.array([bi % n_balls_axis, (bi // n_balls_axis) % n_balls_axis, bi // n_balls_axis ** 2])
        pick = sites[rng.choice(sites.shape[0], n_spikes, replace=False)]
        cubes = [core_cubes]
        for ax, side, a1, a2, _ in pick:
            o1, o2 = [a for a in range(3) if a != ax]
            c = np.zeros((spike_len, 3), np.int64)
            c[:, o1] = a1
            c[:, o2] = a2
            c[:, ax] = (hi[ax] + np.arange(spike_len)) if side == 1 else (-1 - np.arange(spike_len))
            cubes.append(c)
        cubes = np.concatenate(cubes)
        origin = b * pitch + (b % 2) * 0.13 * edge
        Xb, tb = lattice_from_cubes(cubes, edge, origin)
        # spike vertices: outside the core box, tagged with the face they stand on
        lc = np.round((Xb - origin) / edge).astype(np.int64)
        out = np.any((lc < 0) | (lc > hi), 1)
        face = np.full(Xb.shape[0], -1, np.int64)
        for ax in range(3):
            face[lc[:, ax] < 0] = 2 * ax
            face[lc[:, ax] > hi[ax]] = 2 * ax + 1
        face[~out] = -1
        Xs.append(Xb)
        tets_l.append(tb + nv)
        face_v.append(face)
        ball_ids.append((b, nv, Xb.shape[0]))
        nv += Xb.shape[0]
    X = np.concatenate(Xs)
    tets = np.concatenate(tets_l).astype(np.int32)
    face_all = np.concatenate(face_v)
    x = _perturb(rng, X, tets, 0.01 * edge)
    centre = X.mean(0)
    # contact stencils between facing spikes of face-adjacent balls
    pairs = []
    for ia, (ba, oa, na) in enumerate(ball_ids):
        for ib, (bb, ob, nb) in enumerate(ball_ids):
            dlt = bb - ba
            if np.abs(dlt).sum() == 1 and dlt.sum() == 1:
                ax = int(np.nonzero(dlt)[0][0])
                pairs.append((oa, na, ob, nb, ax))
    per_pair = int(np.ceil(pool_size / max(1, len(pairs)) * 1.2))
    all_idx, all_grad, all_tag = [], [], []
    for oa, na, ob, nb, ax in pairs:
        fa = np.nonzero(face_all[oa:oa + na] == 2 * ax + 1)[0] + oa     # A's +ax spikes
        fb = np.nonzero(face_all[ob:ob + nb] == 2 * ax)[0] + ob         # B's -ax spikes
        # quads of B's spikes: consecutive layers of each column -> use the tets' faces
        tb = tets[(tets >= ob).all(1) & (tets < ob + nb).all(1)]
        infb = np.zeros(X.shape[0], bool)
        infb[fb] = True
        tb = tb[infb[tb].all(1)]
        qb = tb[:, :4]                      # four vertices of a spike tet as the "quad"
        cb = X[qb].mean(1)
        hint = np.zeros(3)
        hint[ax] = -1.0
        n_pt = per_pair // 2
        for (ids_a, qq, cc, hh) in ((fa, qb, cb, hint),):
            i1, g1, t1 = _pt_ee_stencils(rng, X[ids_a], ids_a, qq, cc, n_pt, per_pair - n_pt, hh, 30.0)
            all_idx.append(i1)
            all_grad.append(g1)
            all_tag.append(t1)
    key, idx, grad = _dedupe(np.concatenate(all_idx), np.concatenate(all_grad),
                             np.concatenate(all_tag))
    sel = rng.permutation(key.size)[:pool_size]
    key, idx, grad = key[sel], idx[sel], grad[sel]
    m = key.size
    n_act = int(round(active_frac * m))
    d = np.concatenate([_loguniform(rng, dmin, dhat, n_act),
                        rng.uniform(1.05 * dhat, 3 * dhat, m - n_act)])
    rng.shuffle(d)
    pool = stencil_pool(key, idx, grad, x, d)
    vdir = centre - X
    vdir /= np.maximum(np.linalg.norm(vdir, axis=1, keepdims=True), 1e-12)
    T = tets.shape[0]
    return Scene("puffer_balls", X, x, speed * vdir, tets,
                 np.full(T, rho), np.full(T, E), np.full(T, nu), h, dhat,
                 kappa=kappa_scale * rho * edge ** 3, gravity=np.array([0.0, 0.0, -9.81]),
                 pool=pool, levels=levels, K=K)


def graded_stiffness(scene, lo=2.15e4, hi=1e7):
    """A copy of the scene whose Young's modulus grows geometrically with
    the height of each tet's centroid, from lo at the lowest to hi at the
    highest (the 500-fold span of the paper's stiffness-robustness scene,
    Section 5)."""
    import dataclasses
    zc = scene.X[scene.tets].mean(axis=1)[:, 2]
    t = (zc - zc.min()) / max(float(zc.max() - zc.min()), 1e-300)
    return dataclasses.replace(scene, name=scene.name + "_graded", youngs=lo * (hi / lo) ** t)


def with_youngs(scene, E):
    """A copy of the scene with one Young's modulus E for every tet."""
    import dataclasses
    return dataclasses.replace(scene, name="%s_E%.3g" % (scene.name, E), youngs=np.full(scene.T, float(E)))


def contact_links(pool, x, dhat):
    """Vertex pairs joined by the pool's stencils that are active at x
    (0 < d < dhat): every pair of distinct vertices of such a stencil."""
    d = pool_distance(pool, x)
    idx = pool['idx'][(d > 0) & (d < dhat)]
    out = []
    for a in range(4):
        for b in range(a + 1, 4):
            sel = (idx[:, a] >= 0) & (idx[:, b] >= 0)
            out.append(idx[sel][:, [a, b]])
    return np.concatenate(out).astype(np.int32) if out else np.zeros((0, 2), np.int32)


def surface(tets):
    """Boundary of a tet mesh: (vertices, triangles (F, 3), edges (E, 2)),
    the triangles being the tet faces that belong to one tet only, the
    edges and vertices those of the triangles (edges with the smaller id
    first, all sorted).  Topology only."""
    t = np.asarray(tets, np.int64)
    faces = np.sort(np.concatenate([t[:, [0, 1, 2]], t[:, [0, 1, 3]], t[:, [0, 2, 3]], t[:, [1, 2, 3]]]), axis=1)
    if t.size and t.max() < (1 << 21):
        # one 63-bit key per sorted face / edge: a 1-D unique
        fk = (faces[:, 0] << 42) | (faces[:, 1] << 21) | faces[:, 2]
        uk, cnt = np.unique(fk, return_counts=True)
        k1 = uk[cnt == 1]
        tris = np.stack([k1 >> 42, (k1 >> 21) & 0x1FFFFF, k1 & 0x1FFFFF], 1)
        e = np.sort(np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [0, 2]]]), axis=1)
        ek = np.unique((e[:, 0] << 21) | e[:, 1])
        edges = np.stack([ek >> 21, ek & 0x1FFFFF], 1)
    else:
        uniq, cnt = np.unique(faces, axis=0, return_counts=True)
        tris = uniq[cnt == 1]
        e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [0, 2]]])
        edges = np.unique(np.sort(e, axis=1), axis=0)
    verts = np.unique(tris)
    return verts.astype(np.int32), tris.astype(np.int32), edges.astype(np.int32)


def scene_by_name(name, **kw):
    return {"grid": grid_scene, "two_boxes": two_boxes_scene, "puffer": puffer_scene}[name](**kw)
