"""Incremental potential, gradient and SPD-projected Hessian snapshot (FP64).

Test infrastructure (see the package docstring).

Definitions followed:
* E(x) = 1/2 (x - x~)^T M (x - x~) + h^2 Psi(x) + B(x)  (Section 3.1, the
  IPC energy; friction is not part of this path), with
  x~ = x^t + h v^t + h^2 M^-1 f_ext (same equation; f_ext = M g).
* B(x) = kappa * sum_c b(d_c(x)), active only while d_c < dhat (Section 3.1).
  The paper does not print b; this oracle uses the IPC log barrier on the
  unsquared distance, b(d) = -(d - dhat)^2 ln(d / dhat).
* Psi: stable Neo-Hookean (Section 5 names it); this oracle uses the
  rest-stable form Psi(F) = mu/2 (I_C - 3) - mu (J - 1) + lam/2 (J - 1)^2
  with Lame parameters from Young's modulus and Poisson's ratio.
* Contact Hessian projected to k n n^T with k = kappa b''(d), n = grad d
  (Section 4.1, the projected barrier Hessian).  Elastic Hessians are made
  SPD by clamping the eigenvalues of d2Psi/dF2 at zero before mapping with
  dF/dx (the paper requires SPD blocks but does not say how).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


# ------------------------------------------------------------ material

def lame(E, nu):
    E = np.asarray(E, np.float64)
    nu = np.asarray(nu, np.float64)
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def rest_quantities(X, tets, density):
    """Dm^-1 (T,3,3), rest volume (T,), lumped vertex mass (N,)."""
    X = np.asarray(X, np.float64)
    P = X[tets]                                     # (T,4,3)
    Dm = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    Dm_inv = np.linalg.inv(Dm)
    vol = np.linalg.det(Dm) / 6.0
    mass = np.zeros(X.shape[0])
    for j in range(4):
        np.add.at(mass, tets[:, j], density * vol / 4.0)
    return Dm_inv, vol, mass


def inertial_target(x_t, v_t, h, gravity):
    """x~ = x^t + h v^t + h^2 M^-1 f_ext with f_ext = M * gravity."""
    return x_t + h * v_t + h * h * np.asarray(gravity)[None, :]


def deformation_gradient(x, tets, Dm_inv):
    P = np.asarray(x)[tets]
    Ds = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    return Ds @ Dm_inv


# ------------------------------------------------- stable Neo-Hookean

def snh_psi(F, mu, lam):
    Ic = np.einsum('tij,tij->t', F, F)
    J = np.linalg.det(F)
    return 0.5 * mu * (Ic - 3.0) - mu * (J - 1.0) + 0.5 * lam * (J - 1.0) ** 2


def cofactor(F):
    """dJ/dF: columns f1 x f2, f2 x f0, f0 x f1 (f_i = columns of F)."""
    f0, f1, f2 = F[:, :, 0], F[:, :, 1], F[:, :, 2]
    return np.stack([np.cross(f1, f2), np.cross(f2, f0), np.cross(f0, f1)], axis=2)


def snh_P(F, mu, lam):
    """First Piola-Kirchhoff stress dPsi/dF."""
    J = np.linalg.det(F)
    return mu[:, None, None] * F + (lam * (J - 1.0) - mu)[:, None, None] * cofactor(F)


def _skew(a):
    T = a.shape[0]
    S = np.zeros((T, 3, 3))
    S[:, 0, 1], S[:, 0, 2] = -a[:, 2], a[:, 1]
    S[:, 1, 0], S[:, 1, 2] = a[:, 2], -a[:, 0]
    S[:, 2, 0], S[:, 2, 1] = -a[:, 1], a[:, 0]
    return S


def vecF(M):
    """Column-major vectorisation: entry (a,b) -> 3b + a."""
    return np.transpose(M, (0, 2, 1)).reshape(M.shape[0], 9)


def snh_dPdF(F, mu, lam):
    """d2Psi/dF2 as a 9x9 matrix in the column-major vec(F) basis."""
    T = F.shape[0]
    J = np.linalg.det(F)
    g = vecF(cofactor(F))
    f0, f1, f2 = F[:, :, 0], F[:, :, 1], F[:, :, 2]
    HJ = np.zeros((T, 9, 9))
    # d(f1 x f2)/df1 = -[f2]x, d(f1 x f2)/df2 = [f1]x, and cyclic
    HJ[:, 0:3, 3:6] = -_skew(f2)
    HJ[:, 0:3, 6:9] = _skew(f1)
    HJ[:, 3:6, 0:3] = _skew(f2)
    HJ[:, 3:6, 6:9] = -_skew(f0)
    HJ[:, 6:9, 0:3] = -_skew(f1)
    HJ[:, 6:9, 3:6] = _skew(f0)
    H = mu[:, None, None] * np.eye(9)[None] + lam[:, None, None] * g[:, :, None] * g[:, None, :] \
        + (lam * (J - 1.0) - mu)[:, None, None] * HJ
    return H


def psd_project(H):
    """Clamp the eigenvalues of symmetric matrices at zero (a matrix
    function, so the result is unique even with repeated eigenvalues)."""
    w, V = np.linalg.eigh(H)
    return np.einsum('tij,tj,tkj->tik', V, np.maximum(w, 0.0), V)


def dFdx(Dm_inv):
    """B = d vec(F) / d x_e (T,9,12) for x_e = (x0,x1,x2,x3) flattened."""
    T = Dm_inv.shape[0]
    coef = np.zeros((T, 4, 3))                  # coef[t, j, b] = dF_{ab}/dx_{j,a}
    coef[:, 1:, :] = Dm_inv
    coef[:, 0, :] = -Dm_inv.sum(axis=1)
    B = np.zeros((T, 9, 12))
    for b in range(3):
        for a in range(3):
            for j in range(4):
                B[:, 3 * b + a, 3 * j + a] = coef[:, j, b]
    return B


def elem_hessians(x, tets, Dm_inv, vol, mu, lam, h, project=True):
    """12x12 Hessians of h^2 V_e Psi(F_e) w.r.t. the four vertex positions."""
    F = deformation_gradient(x, tets, Dm_inv)
    Hf = snh_dPdF(F, mu, lam)
    if project:
        Hf = psd_project(Hf)
    B = dFdx(Dm_inv)
    return (h * h * vol)[:, None, None] * np.einsum('tai,tab,tbj->tij', B, Hf, B)


def elastic_energy(x, tets, Dm_inv, vol, mu, lam):
    F = deformation_gradient(x, tets, Dm_inv)
    return float(np.sum(vol * snh_psi(F, mu, lam)))


def elastic_gradient(x, tets, Dm_inv, vol, mu, lam):
    """d/dx of sum_e V_e Psi(F_e), shape (N,3)."""
    F = deformation_gradient(x, tets, Dm_inv)
    G = vol[:, None, None] * snh_P(F, mu, lam) @ np.transpose(Dm_inv, (0, 2, 1))
    g = np.zeros_like(np.asarray(x, np.float64))
    for j in range(3):
        np.add.at(g, tets[:, j + 1], G[:, :, j])
    np.add.at(g, tets[:, 0], -G.sum(axis=2))
    return g


# ---------------------------------------------------------- barrier

def barrier(d, dhat):
    """b, b', b'' of the log barrier; zero outside (0, dhat)."""
    d = np.asarray(d, np.float64)
    act = (d > 0) & (d < dhat)
    b = np.zeros_like(d)
    b1 = np.zeros_like(d)
    b2 = np.zeros_like(d)
    da = d[act]
    r = da - dhat
    L = np.log(da / dhat)
    b[act] = -r * r * L
    b1[act] = -2.0 * r * L - r * r / da
    b2[act] = -2.0 * L - 4.0 * r / da + r * r / (da * da)
    return b, b1, b2


def stencil_gather(idx, x):
    """(m,12) stencil positions, zero in padded slots."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    return np.where(idx[..., None] >= 0, x[np.maximum(idx, 0)], 0.0).reshape(-1, 12)


def stencil_scatter(idx, vals, N):
    """Add (m,12) per-stencil vectors into an (N,3) array."""
    out = np.zeros((N, 3))
    v = vals.reshape(-1, 4, 3)
    for j in range(4):
        ok = idx[:, j] >= 0
        np.add.at(out, idx[ok, j], v[ok, j])
    return out


# ------------------------------------------------------------- scene

class Problem:
    """Static data of one scene: mesh, materials, time-step constants."""

    def __init__(self, scene):
        self.N = scene.X.shape[0]
        self.tets = np.asarray(scene.tets, np.int64)
        self.Dm_inv, self.vol, self.mass = rest_quantities(scene.X, self.tets, scene.density)
        self.mu, self.lam = lame(scene.youngs, scene.poisson)
        self.h = float(scene.h)
        self.dhat = float(scene.dhat)
        self.kappa = float(scene.kappa)
        self.gravity = np.asarray(scene.gravity, np.float64)

    # energy and gradient ------------------------------------------------
    def energy(self, x, x_tilde, cset):
        x = np.asarray(x, np.float64).reshape(-1, 3)
        dx = x - x_tilde.reshape(-1, 3)
        Ein = 0.5 * float(np.sum(self.mass[:, None] * dx * dx))
        Eel = self.h ** 2 * elastic_energy(x, self.tets, self.Dm_inv, self.vol, self.mu, self.lam)
        d = cset['d']
        if np.any(d <= 0):
            return np.inf
        b, _, _ = barrier(d, self.dhat)
        return Ein + Eel + self.kappa * float(np.sum(b))

    def gradient(self, x, x_tilde, cset):
        x = np.asarray(x, np.float64).reshape(-1, 3)
        g = self.mass[:, None] * (x - x_tilde.reshape(-1, 3))
        g += self.h ** 2 * elastic_gradient(x, self.tets, self.Dm_inv, self.vol, self.mu, self.lam)
        _, b1, _ = barrier(cset['d'], self.dhat)
        g += stencil_scatter(cset['idx'], (self.kappa * b1)[:, None] * cset['grad'], self.N)
        return g.reshape(-1)

    # Hessian snapshot --------------------------------------------------
    def contact_stiffness(self, d):
        _, _, b2 = barrier(d, self.dhat)
        return self.kappa * b2

    def elastic_hessians(self, x, project=True):
        return elem_hessians(np.asarray(x, np.float64).reshape(-1, 3), self.tets, self.Dm_inv,
                             self.vol, self.mu, self.lam, self.h, project)

    def assemble(self, x_base, cset_base, project=True):
        """Sparse H_base = M + sum_e S_e^T H_e S_e + sum_c k_c n_c n_c^T."""
        N = self.N
        He = self.elastic_hessians(x_base, project)
        dof = (3 * self.tets[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
        rows = np.repeat(dof, 12, axis=1).reshape(-1)
        cols = np.tile(dof, (1, 12)).reshape(-1)
        H = sp.coo_matrix((He.reshape(-1), (rows, cols)), shape=(3 * N, 3 * N)).tocsr()
        H = H + sp.diags(np.repeat(self.mass, 3))
        H = H + contact_outer(cset_base['idx'], cset_base['grad'],
                              self.contact_stiffness(cset_base['d']), N)
        return H.tocsr()


def contact_outer(idx, grad, k, N):
    """Sparse sum_c k_c n_c n_c^T for stencils (idx, grad=n)."""
    m = idx.shape[0]
    if m == 0:
        return sp.csr_matrix((3 * N, 3 * N))
    dof = (3 * np.maximum(idx, 0)[:, :, None] + np.arange(3)[None, None, :]).reshape(m, 12)
    valid = np.repeat(idx >= 0, 3, axis=1)
    vals = k[:, None, None] * grad[:, :, None] * grad[:, None, :]
    vals = vals * (valid[:, :, None] & valid[:, None, :])
    rows = np.repeat(dof, 12, axis=1).reshape(-1)
    cols = np.tile(dof, (1, 12)).reshape(-1)
    return sp.coo_matrix((vals.reshape(-1), (rows, cols)), shape=(3 * N, 3 * N)).tocsr()


def update_matrix(idx, u, N):
    """Sparse U (3N x m) whose columns are the stencil vectors u (m,12)."""
    m = idx.shape[0]
    dof = (3 * np.maximum(idx, 0)[:, :, None] + np.arange(3)[None, None, :]).reshape(m, 12)
    valid = np.repeat(idx >= 0, 3, axis=1)
    cols = np.repeat(np.arange(m), 12).reshape(m, 12)
    v = np.where(valid, u, 0.0)
    return sp.coo_matrix((v[valid], (dof[valid], cols[valid])), shape=(3 * N, m)).tocsr()
