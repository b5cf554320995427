"""Python binding of the C ABI: argument marshalling only.

PyTorch provides device memory and the stream; every computation runs in
the HIP library.  Vectors live in the library's Morton vertex order; the
helpers ``to_lib`` / ``from_lib`` move host arrays in and out of it.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _abi
from ._abi import MasConfig, MasContacts, MasMesh, MasStepOut, check


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def make_config(scene=None, levels=None, K=None, block_prec="f64", coarse_prec=None,
                hess_prec=None, delta=0.3, cos_rot=None, eps_sing=1e-12, prec_guard=None,
                deterministic=False, max_contacts=0, max_tris=0, max_edges=0, precond="mas", hierarchy="morton"):
    cfg = MasConfig()
    _abi.lib().mas_default_config(ctypes.byref(cfg))
    if scene is not None:
        cfg.kappa = float(scene.kappa)
        cfg.dhat = float(scene.dhat)
        cfg.h = float(scene.h)
        for a in range(3):
            cfg.gravity[a] = float(scene.gravity[a])
        cfg.num_levels = int(levels if levels is not None else scene.levels)
        cfg.max_rank = int(K if K is not None else scene.K)
    else:
        if levels is not None:
            cfg.num_levels = int(levels)
        if K is not None:
            cfg.max_rank = int(K)
    cfg.block_prec = _abi.PREC[block_prec]
    cp = coarse_prec or "f64"
    hp = hess_prec or ("f64" if block_prec == "f64" else "f32")
    cfg.coarse_prec = _abi.PREC[cp]
    cfg.hess_prec = _abi.PREC[hp]
    cfg.restart_delta = float(delta)
    cfg.eps_sing = float(eps_sing)
    if cos_rot is not None:
        cfg.cos_rot = float(cos_rot)
    if prec_guard is not None:
        cfg.prec_guard = float(prec_guard)
    cfg.deterministic = int(bool(deterministic))
    cfg.max_contacts = int(max_contacts)
    cfg.max_tris = int(max_tris)
    cfg.max_edges = int(max_edges)
    cfg.precond = _abi.PRECOND[precond]
    cfg.hierarchy = _abi.HIERARCHY[hierarchy]
    return cfg


class DeviceContacts:
    """Contact stencils on the device in library vertex numbering."""

    def __init__(self, key, idx, grad, d=None, off=None, device="cuda"):
        self.key = torch.as_tensor(np.ascontiguousarray(key).view(np.int64), device=device)
        self.idx = torch.as_tensor(np.ascontiguousarray(idx, np.int32), device=device)
        self.grad = torch.as_tensor(np.ascontiguousarray(grad, np.float64), device=device)
        m = self.key.shape[0]
        self.d = (torch.as_tensor(np.ascontiguousarray(d, np.float64), device=device) if d is not None
                  else torch.zeros(m, dtype=torch.float64, device=device))
        self.off = (torch.as_tensor(np.ascontiguousarray(off, np.float64), device=device)
                    if off is not None else None)

    @classmethod
    def from_tensors(cls, key, idx, grad, d):
        """A view of device tensors (no copies)."""
        c = cls.__new__(cls)
        c.key, c.idx, c.grad, c.d, c.off = key, idx, grad, d, None
        return c

    @property
    def m(self):
        return int(self.key.shape[0])

    def struct(self):
        c = MasContacts()
        c.m = self.m
        c.key = self.key.data_ptr() if self.m else None
        c.idx = self.idx.data_ptr() if self.m else None
        c.d = self.d.data_ptr() if self.m else None
        c.grad = self.grad.data_ptr() if self.m else None
        return c


def vertex_order(X, tets, levels, hierarchy="morton", links=None):
    """mas_vertex_order: perm[new] = old vertex id of the hierarchy's order
    (host only); ``links`` (k, 2) vertex pairs joined by contacts."""
    X = np.ascontiguousarray(X, np.float64)
    tets = np.ascontiguousarray(tets, np.int32)
    lk = np.ascontiguousarray(np.zeros((0, 2)) if links is None else links, np.int32)
    mesh = MasMesh()
    mesh.num_vertices = X.shape[0]
    mesh.num_tets = tets.shape[0]
    mesh.rest_x = X.ctypes.data
    mesh.tets = tets.ctypes.data
    mesh.num_links = lk.shape[0]
    mesh.links = lk.ctypes.data if lk.shape[0] else None
    perm = np.zeros(X.shape[0], np.int32)
    check("mas_vertex_order", _abi.lib().mas_vertex_order(ctypes.byref(mesh), int(levels),
                                                          _abi.HIERARCHY[hierarchy], perm.ctypes.data))
    return perm


class MasContext:
    """One library context for one mesh (``mas_create`` .. ``mas_destroy``)."""

    def __init__(self, scene, cfg, device="cuda", links=None, scene_offsets=None):
        L = _abi.lib()
        self.device = device
        self.scene = scene
        X = np.ascontiguousarray(scene.X, np.float64)
        tets = np.ascontiguousarray(scene.tets, np.int32)
        lk = np.ascontiguousarray(np.zeros((0, 2)) if links is None else links, np.int32)
        so = np.ascontiguousarray(np.array([0, X.shape[0]]) if scene_offsets is None else scene_offsets, np.int64)
        self._host = [X, tets, np.ascontiguousarray(scene.density, np.float64),
                      np.ascontiguousarray(scene.youngs, np.float64),
                      np.ascontiguousarray(scene.poisson, np.float64), lk, so]
        mesh = MasMesh()
        mesh.num_vertices = X.shape[0]
        mesh.num_tets = tets.shape[0]
        mesh.rest_x = X.ctypes.data
        mesh.tets = tets.ctypes.data
        mesh.density = self._host[2].ctypes.data
        mesh.youngs = self._host[3].ctypes.data
        mesh.poisson = self._host[4].ctypes.data
        mesh.num_links = lk.shape[0]
        mesh.links = lk.ctypes.data if lk.shape[0] else None
        mesh.num_scenes = so.shape[0] - 1
        mesh.scene_offsets = so.ctypes.data
        self.N = X.shape[0]
        self.perm = np.zeros(self.N, np.int32)
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream().cuda_stream
        check("mas_create", L.mas_create(ctypes.byref(cfg), ctypes.byref(mesh), ctypes.c_void_p(stream),
                                         ctypes.byref(h), self.perm.ctypes.data))
        self.h = h
        self.cfg = cfg
        self.rank = np.empty(self.N, np.int64)
        self.rank[self.perm] = np.arange(self.N)
        nsub = np.zeros(6, np.int64)
        levels = ctypes.c_int32()
        check("mas_query", L.mas_query(h, None, None, ctypes.byref(levels), nsub.ctypes.data))
        self.levels = levels.value
        self.nsub = nsub[:self.levels].copy()
        self.out = torch.zeros(ctypes.sizeof(MasStepOut) // 8, dtype=torch.float64, device=device)

    def close(self):
        if self.h:
            _abi.lib().mas_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------- marshalling
    def to_lib(self, v):
        """(N,3) or (3N,) host array in original order -> (3N,) device tensor."""
        a = np.asarray(v, np.float64).reshape(-1, 3)[self.perm].reshape(-1)
        return torch.as_tensor(np.ascontiguousarray(a), device=self.device)

    def from_lib(self, t):
        """(3N,) device tensor or host array in library order -> (3N,) host
        array in original order."""
        a = (t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)).reshape(-1, 3)
        out = np.empty_like(a)
        out[self.perm] = a
        return out.reshape(-1)

    def contacts(self, cset, sort=False):
        """Host contact set (original vertex ids) -> DeviceContacts in library
        numbering; ``sort`` orders the stencils by their smallest library
        vertex, which keeps the library's scatter kernels local."""
        idx = np.where(cset['idx'] >= 0, self.rank[np.maximum(cset['idx'], 0)], -1).astype(np.int32)
        order = slice(None)
        if sort:
            vmin = np.where(idx >= 0, idx, np.iinfo(np.int32).max).min(axis=1)
            order = np.argsort(vmin, kind='stable')
        pick = (lambda a: None if a is None else np.ascontiguousarray(a[order]))
        return DeviceContacts(cset['key'][order], idx[order], cset['grad'][order], d=pick(cset.get('d')),
                              off=pick(cset.get('off')), device=self.device)

    def vec(self):
        return torch.zeros(3 * self.N, dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------- calls
    def build(self, x, base):
        c = base.struct() if base is not None else None
        check("mas_build", _abi.lib().mas_build(self.h, _ptr(x), ctypes.byref(c) if c else None))

    def woodbury_update(self, curr, rank_hist=None):
        c = curr.struct()
        check("mas_woodbury_update", _abi.lib().mas_woodbury_update(self.h, ctypes.byref(c), _ptr(rank_hist)))

    def apply(self, g, z=None):
        z = self.vec() if z is None else z
        check("mas_apply", _abi.lib().mas_apply(self.h, _ptr(g), _ptr(z)))
        return z

    def hess_vec(self, v, with_update=True, y=None):
        y = self.vec() if y is None else y
        check("hess_vec", _abi.lib().hess_vec(self.h, _ptr(v), _ptr(y), int(with_update)))
        return y

    def subspace_step(self, g, z, z_prev, vz, p, vp, restart):
        check("pncg_subspace_step", _abi.lib().pncg_subspace_step(
            self.h, _ptr(g), _ptr(z), _ptr(z_prev), _ptr(vz), _ptr(p), _ptr(vp), int(restart),
            _ptr(self.out)))
        return self.out

    def subspace_step_noalloc(self, g, z, z_prev, vz, p, vp, restart, out=None):
        """pncg_subspace_step_noalloc: the subspace step with the library's
        fixed device workspace (no allocation)."""
        out = self.out if out is None else out
        check("pncg_subspace_step_noalloc", _abi.lib().pncg_subspace_step_noalloc(
            self.h, _ptr(g), _ptr(z), _ptr(z_prev), _ptr(vz), _ptr(p), _ptr(vp), int(restart), _ptr(out)))
        return out

    def beta_step(self, rule, g, g_prev, z, z_prev, vz, d, vd, restart, p):
        """pncg_beta_step: a comparison direction rule ("fr", "cd", "dk");
        d, vd in/out, p the step; the step scalars land in self.out (alpha
        in mu, beta in nu)."""
        check("pncg_beta_step", _abi.lib().pncg_beta_step(
            self.h, _abi.BETA[rule], _ptr(g), _ptr(g_prev), _ptr(z), _ptr(z_prev), _ptr(vz), _ptr(d), _ptr(vd),
            int(restart), _ptr(p), _ptr(self.out)))
        return self.out

    def scenes(self):
        """(number of scenes, library vertex offset of each scene)."""
        S = ctypes.c_int32()
        check("mas_scenes", _abi.lib().mas_scenes(self.h, ctypes.byref(S), None))
        voff = np.zeros(S.value + 1, np.int64)
        check("mas_scenes", _abi.lib().mas_scenes(self.h, None, voff.ctypes.data))
        return S.value, voff

    def subspace_step_scenes(self, g, z, z_prev, vz, p, vp, restart, out):
        """pncg_subspace_step_scenes: restart (device int32, one per scene),
        out (device float64, one MasStepOut per scene)."""
        check("pncg_subspace_step_scenes", _abi.lib().pncg_subspace_step_scenes(
            self.h, _ptr(g), _ptr(z), _ptr(z_prev), _ptr(vz), _ptr(p), _ptr(vp), _ptr(restart), _ptr(out)))

    def energy_grad_scenes(self, x, x_tilde, contacts, E, g=None):
        c = contacts.struct() if contacts is not None else None
        check("mas_energy_grad_scenes", _abi.lib().mas_energy_grad_scenes(
            self.h, _ptr(x), _ptr(x_tilde), ctypes.byref(c) if c else None, _ptr(E), _ptr(g)))

    def step_scenes(self, x, p, scale, x_out):
        check("mas_step_scenes", _abi.lib().mas_step_scenes(self.h, _ptr(x), _ptr(p), _ptr(scale), _ptr(x_out)))

    def step_out(self, out=None):
        """The step scalars (from self.out, or from a copy of it, device or
        host)."""
        src = self.out if out is None else out
        arr = src if isinstance(src, np.ndarray) else src.cpu().numpy()
        raw = np.ascontiguousarray(arr, np.float64).view(np.uint8)
        s = MasStepOut.from_buffer_copy(raw.tobytes())
        return {f: getattr(s, f) for f in _abi.STEP_FIELDS}

    def energy_grad(self, x, x_tilde, contacts, E, g=None):
        c = contacts.struct() if contacts is not None else None
        check("mas_energy_grad", _abi.lib().mas_energy_grad(self.h, _ptr(x), _ptr(x_tilde),
                                                           ctypes.byref(c) if c else None, _ptr(E), _ptr(g)))

    def next_frame(self, x_new, x_old, v=None, x_tilde=None):
        check("mas_next_frame", _abi.lib().mas_next_frame(self.h, _ptr(x_new), _ptr(x_old), _ptr(v), _ptr(x_tilde)))

    def inertial_target(self, x_t, v_t, out=None):
        out = self.vec() if out is None else out
        check("mas_inertial_target", _abi.lib().mas_inertial_target(self.h, _ptr(x_t), _ptr(v_t), _ptr(out)))
        return out

    def stencil_distance(self, x, contacts):
        check("mas_stencil_distance", _abi.lib().mas_stencil_distance(
            self.h, _ptr(x), contacts.m, _ptr(contacts.idx), _ptr(contacts.grad), _ptr(contacts.off),
            _ptr(contacts.d)))

    def ccd_steps(self, x, p, pairs, kind, dist, alpha_pair=None, alpha=None):
        """Conservative CCD step of each point-triangle / edge-edge pair and
        the per-subdomain minima (device tensors; pairs in library ids)."""
        m = int(pairs.shape[0])
        check("mas_ccd_steps", _abi.lib().mas_ccd_steps(self.h, _ptr(x), _ptr(p), m, _ptr(pairs), _ptr(kind),
                                                       _ptr(dist), _ptr(alpha_pair), _ptr(alpha)))

    def contact_distances(self, x, pairs, kind, dist, grad=None, type=None):
        """Distance, gradient and closest-feature type of each point-triangle
        / edge-edge pair (device tensors; pairs in library ids)."""
        m = int(pairs.shape[0])
        check("mas_contact_distances", _abi.lib().mas_contact_distances(
            self.h, _ptr(x), m, _ptr(pairs), _ptr(kind), _ptr(dist), _ptr(grad), _ptr(type)))

    def constraint_set(self, x, verts, tris, edges, dhat, pairs, kind, dist, grad=None, key=None):
        """Active point-triangle / edge-edge pairs within dhat (device
        tensors in library ids; outputs of capacity pairs.shape[0]).
        Returns the number of pairs found (may exceed the capacity)."""
        cnt = ctypes.c_int64(0)
        check("mas_constraint_set", _abi.lib().mas_constraint_set(
            self.h, _ptr(x), float(dhat), int(verts.shape[0]), _ptr(verts), int(tris.shape[0]), _ptr(tris),
            int(edges.shape[0]), _ptr(edges), int(pairs.shape[0]), _ptr(pairs), _ptr(kind), _ptr(dist), _ptr(grad),
            _ptr(key), ctypes.byref(cnt)))
        return int(cnt.value)

    def safe_step(self, x, p, cand, scale, x_out, alpha=None):
        c = cand.struct() if cand is not None else None
        check("mas_safe_step", _abi.lib().mas_safe_step(self.h, _ptr(x), _ptr(p), ctypes.byref(c) if c else None,
                                                       float(scale), _ptr(alpha), _ptr(x_out)))

    def ccd_safe_step(self, x, p, radius, pairs, kind, dist, m, scale, x_out, alpha=None):
        """Per-subdomain CCD steps over m candidate pairs within radius, the
        mixed-step damping rounds, and x_out = x + scale alpha p."""
        check("mas_ccd_safe_step", _abi.lib().mas_ccd_safe_step(
            self.h, _ptr(x), _ptr(p), float(radius), int(m), _ptr(pairs), _ptr(kind), _ptr(dist), float(scale),
            _ptr(alpha), _ptr(x_out)))

    def stats(self):
        """Counters of the last Woodbury update and safe step (synchronises)."""
        st = _abi.MasIterStats()
        check("mas_read_stats", _abi.lib().mas_read_stats(self.h, ctypes.byref(st)))
        out = {f: getattr(st, f) for f, _ in _abi.MasIterStats._fields_ if f != "alpha_hist"}
        out["alpha_hist"] = list(st.alpha_hist)
        return out

    def sync(self):
        buf = ctypes.create_string_buffer(256)
        code = _abi.lib().mas_sync_status(self.h, buf, 256)
        return code, buf.value.decode()

    def get_block(self, level, d):
        out = np.zeros((96, 96))
        check("mas_get_block", _abi.lib().mas_get_block(self.h, int(level), int(d), out.ctypes.data))
        return out

    def profile(self, enable=True, timers=None):
        """Enables the kernel timers (all, or only the named ones)."""
        mask = 0xffffffff if timers is None else sum(1 << _abi.TIMERS[t] for t in timers)
        check("mas_profile_select", _abi.lib().mas_profile_select(self.h, mask))
        check("mas_profile_enable", _abi.lib().mas_profile_enable(self.h, int(enable)))

    def profile_read(self, timer):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        check("mas_profile_read", _abi.lib().mas_profile_read(self.h, _abi.TIMERS[timer], ctypes.byref(ms),
                                                             ctypes.byref(n)))
        return ms.value, n.value

    def block_precisions(self, level=0):
        """Blocks of a level stored as {f64, f32, bf16, f16} by the last build."""
        counts = np.zeros(4, np.int64)
        check("mas_block_precisions", _abi.lib().mas_block_precisions(self.h, int(level), counts.ctypes.data))
        return dict(zip(("f64", "f32", "bf16", "f16"), counts.tolist()))

    def get_selection(self):
        D0 = int(self.nsub[0])
        K = max(int(self.cfg.max_rank), 0)
        rank = np.zeros(D0, np.int32)
        sel = np.full(D0 * max(K, 1), -1, np.int32)
        check("mas_get_selection", _abi.lib().mas_get_selection(self.h, rank.ctypes.data, sel.ctypes.data))
        return rank, sel[:D0 * K].reshape(D0, K)
