"""Multilevel additive Schwarz preconditioner from its definition (FP64).

Test infrastructure (see the package docstring).

Definitions followed (Section 3.3 and supplement Section 1):
* level 0: M_(0)^-1 = sum_d S_d^T (S_d A S_d^T)^-1 S_d over non-overlapping
  subdomains (supplement Eqs. (1)-(2));
* coarse levels: A_(l) = C_(l) A C_(l)^T with binary C_(l) (supplement
  Eq. (3)); M_(l)^-1 is additive Schwarz on A_(l), i.e. the block-diagonal
  inverse over the level-l subdomains;
* P = M_(0)^-1 + sum_l C_(l)^T M_(l)^-1 C_(l) (supplement Eq. (4)).

Readings where the paper leaves the choice open (the grouping the paper
describes is connectivity-aware; the Morton grouping is the alternative
it names in supplement Section 1.2):
* vertices are ordered by a 63-bit Morton code of their rest positions
  (21 bits per axis, positions normalised to the scene's bounding box),
  stable-sorted so ties keep the original order;
* a level-l node is a run of 32^l consecutive vertices in that order; every
  node keeps three DOFs (x, y, z), so C_(l) is the binary node-membership
  matrix Kronecker I_3;
* a level-l subdomain is a run of 32 consecutive level-l nodes (96x96
  blocks); the last one may be smaller.

Every block is cut out of the assembled matrix with explicit S_d / C_(l)
and inverted with numpy.linalg.inv; nothing is blocked or fused.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SUB = 32  # vertices (or nodes) per subdomain


def morton_codes(X):
    X = np.asarray(X, np.float64)
    lo = X.min(axis=0)
    hi = X.max(axis=0)
    ext = hi - lo
    ext = np.where(ext > 0, ext, 1.0)
    q = np.floor((X - lo) / ext * 2097151.0)
    q = np.clip(q, 0, 2097151).astype(np.uint64)
    code = np.zeros(X.shape[0], dtype=np.uint64)
    for b in range(21):
        for a in range(3):
            bit = (q[:, a] >> np.uint64(b)) & np.uint64(1)
            code |= bit << np.uint64(3 * b + a)
    return code


def morton_perm(X):
    """perm[new] = old vertex id, sorted by Morton code, ties by id."""
    return np.argsort(morton_codes(X), kind='stable').astype(np.int64)


class Hierarchy:
    """Subdomain and coarsening structure for N vertices and L levels."""

    def __init__(self, X, levels):
        self.N = X.shape[0]
        self.L = levels
        self.perm = morton_perm(X)
        self.rank = np.empty(self.N, np.int64)
        self.rank[self.perm] = np.arange(self.N)

    def subdomain_of_vertex(self, v):
        return self.rank[v] // SUB

    def num_subdomains(self, level=0):
        nodes = self.N
        for _ in range(level):
            nodes = -(-nodes // SUB)
        return -(-nodes // SUB)

    def num_nodes(self, level):
        nodes = self.N
        for _ in range(level):
            nodes = -(-nodes // SUB)
        return nodes

    def subdomain_dofs(self, d):
        """Original-order DOF indices selected by S_d (level 0)."""
        verts = self.perm[SUB * d: min(SUB * (d + 1), self.N)]
        return (3 * verts[:, None] + np.arange(3)[None, :]).reshape(-1)

    def S(self, d):
        dofs = self.subdomain_dofs(d)
        n = dofs.size
        return sp.coo_matrix((np.ones(n), (np.arange(n), dofs)), shape=(n, 3 * self.N)).tocsr()

    def C(self, level):
        """Binary coarsening matrix C_(l) (3 N_l x 3 N)."""
        node = self.rank // (SUB ** level)
        Nl = self.num_nodes(level)
        rows = (3 * node[:, None] + np.arange(3)[None, :]).reshape(-1)
        cols = (3 * np.arange(self.N)[:, None] + np.arange(3)[None, :]).reshape(-1)
        return sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(3 * Nl, 3 * self.N)).tocsr()


class MAS:
    """P built from an assembled SPD matrix A at every level."""

    def __init__(self, hier, A):
        self.h = hier
        A = sp.csr_matrix(A)
        self.fine = []
        for d in range(hier.num_subdomains(0)):
            dofs = hier.subdomain_dofs(d)
            blk = A[dofs][:, dofs].toarray()
            self.fine.append(np.linalg.inv(blk))
        self.base_blocks = None
        self.coarse = []
        for l in range(1, hier.L):
            Cl = hier.C(l)
            Al = (Cl @ A @ Cl.T).tocsr()
            n_nodes = hier.num_nodes(l)
            invs = []
            for dd in range(-(-n_nodes // SUB)):
                nd = np.arange(SUB * dd, min(SUB * (dd + 1), n_nodes))
                dofs = (3 * nd[:, None] + np.arange(3)[None, :]).reshape(-1)
                invs.append((dofs, np.linalg.inv(Al[dofs][:, dofs].toarray())))
            self.coarse.append((Cl, Al, invs))

    def apply_level0(self, g, blocks=None):
        blocks = self.fine if blocks is None else blocks
        z = np.zeros_like(g)
        for d, Binv in enumerate(blocks):
            dofs = self.h.subdomain_dofs(d)
            z[dofs] += Binv @ g[dofs]
        return z

    def apply_coarse(self, g):
        z = np.zeros_like(g)
        for Cl, _, invs in self.coarse:
            r = Cl @ g
            c = np.zeros_like(r)
            for dofs, Minv in invs:
                c[dofs] = Minv @ r[dofs]
            z += Cl.T @ c
        return z

    def apply(self, g, blocks=None):
        """z = P g with the given (possibly updated) level-0 inverses."""
        g = np.asarray(g, np.float64)
        return self.apply_level0(g, blocks) + self.apply_coarse(g)

    def dense(self, blocks=None):
        n = 3 * self.h.N
        return np.stack([self.apply(e, blocks) for e in np.eye(n)], axis=1)
