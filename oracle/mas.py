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

The connectivity-aware grouping (supplement Section 1.2: an adjacency
graph of nodes that share an element, grouped by greedy aggregation) is
the alternative order ``connectivity_perm``; the paper gives no procedure,
and the reading taken here is:
* level-0 graph: vertices adjacent when they share a tet or are joined by
  a contact link (the paper's reconnection: primitives in close proximity
  join the graph; taken once, from the contacts when the hierarchy is
  built); its nodes are numbered component by component (components in
  the order of their smallest Morton rank), by Morton rank inside a
  component;
* a cluster starts at the smallest unassigned node and repeatedly takes the
  smallest unassigned node adjacent to any of its members, or, when there
  is none, the smallest unassigned node, until it holds 32 nodes;
  clusters are numbered in the order they are started;
* the graph of level l + 1 has the clusters of level l as nodes, adjacent
  when some of their members are, and is aggregated the same way;
* a node holding fewer than 32^l vertices (only the last one can) is kept
  out of the growth and appended to the last cluster (or starts one of its
  own when that cluster is full), so every level-l node but the last holds
  exactly 32^l vertices;
* the vertex order lists the clusters of the top level in their order and,
  inside each cluster, its members in the order they were added, down to
  the vertices; runs of 32^l consecutive vertices are then the level-l
  nodes, as for the Morton order.
Reconnecting again as contacts form later would change the order, and
with it the data layout, between rebuilds; it is not part of this reading.

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


def vertex_adjacency(tets, n, links=None):
    """Adjacency sets of the graph whose nodes 0..n-1 are adjacent when they
    share a tet or form a link (both given in those node ids)."""
    adj = [set() for _ in range(n)]
    for t in np.asarray(tets, np.int64).reshape(-1, 4):
        for a in range(4):
            for b in range(4):
                if t[a] != t[b]:
                    adj[int(t[a])].add(int(t[b]))
    if links is not None:
        for a, b in np.asarray(links, np.int64).reshape(-1, 2):
            if a != b:
                adj[int(a)].add(int(b))
                adj[int(b)].add(int(a))
    return adj


def aggregate(adj, n, sub=SUB, partial_last=False):
    """Greedy aggregation of the nodes 0..n-1 of a graph into clusters of
    ``sub`` nodes (the reading in the module docstring).  With
    ``partial_last`` the node n-1 is left out of the growth and appended to
    the last cluster (or starts its own).  Returns the clusters, each the
    list of its nodes in the order they were added."""
    limit = n - 1 if partial_last else n
    assigned = np.zeros(n, bool)
    clusters = []
    for seed in range(limit):
        if assigned[seed]:
            continue
        members = []
        cand = set()
        u = seed
        while True:
            members.append(u)
            assigned[u] = True
            cand.discard(u)
            cand.update(w for w in adj[u] if w < limit and not assigned[w])
            if len(members) == sub:
                break
            if cand:
                u = min(cand)
            else:
                rest = np.flatnonzero(~assigned[:limit])
                if rest.size == 0:
                    break
                u = int(rest[0])
        clusters.append(members)
    if partial_last:
        if clusters and len(clusters[-1]) < sub:
            clusters[-1].append(n - 1)
        else:
            clusters.append([n - 1])
    return clusters


def cluster_adjacency(adj, clusters):
    """Adjacency of the clusters: two are adjacent when some of their
    members are."""
    cid = np.empty(len(adj), np.int64)
    for c, mem in enumerate(clusters):
        cid[mem] = c
    cadj = [set() for _ in clusters]
    for u, nb in enumerate(adj):
        for w in nb:
            if cid[u] != cid[w]:
                cadj[cid[u]].add(int(cid[w]))
    return cadj


def component_major_perm(X, tets, links=None):
    """perm[id] = vertex of level-0 node id: vertices grouped by connected
    component of the graph of tets and links (components in the order of
    their smallest Morton rank), by Morton rank inside a component."""
    from scipy.sparse.csgraph import connected_components
    N = X.shape[0]
    mperm = morton_perm(X)
    t = np.asarray(tets, np.int64)
    rows = np.repeat(t, 4, axis=1).ravel()
    cols = np.tile(t, (1, 4)).ravel()
    if links is not None:
        lk = np.asarray(links, np.int64).reshape(-1, 2)
        rows = np.concatenate([rows, lk[:, 0]])
        cols = np.concatenate([cols, lk[:, 1]])
    A = sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(N, N)).tocsr()
    _, lab = connected_components(A, directed=False)
    comp = lab[mperm]                      # component of each Morton rank
    first = np.full(comp.max() + 1 if N else 0, N, np.int64)
    np.minimum.at(first, comp, np.arange(N))
    order = np.lexsort((np.arange(N), first[comp]))
    return mperm[order]


def connectivity_clusters(X, tets, levels, sub=SUB, links=None):
    """The clusters of every level (level l: clusters of level-l nodes) and
    the vertex of each level-0 node."""
    N = X.shape[0]
    mperm = component_major_perm(X, tets, links)
    mrank = np.empty(N, np.int64)
    mrank[mperm] = np.arange(N)
    adj = vertex_adjacency(mrank[np.asarray(tets, np.int64)], N,
                           None if links is None else mrank[np.asarray(links, np.int64)])
    size = np.ones(N, np.int64)
    out = []
    for l in range(levels):
        n = len(adj)
        partial = n > 0 and size[-1] < sub ** l
        cl = aggregate(adj, n, sub, partial_last=partial)
        out.append(cl)
        size = np.array([size[m].sum() for m in cl], np.int64)
        adj = cluster_adjacency(adj, cl)
    return mperm, out


def connectivity_perm(X, tets, levels, sub=SUB, links=None):
    """perm[new] = old vertex id of the connectivity-aware order."""
    mperm, cls = connectivity_clusters(X, tets, levels, sub, links)

    def expand(l, c):
        if l < 0:
            return [c]
        out = []
        for m in cls[l][c]:
            out.extend(expand(l - 1, m))
        return out

    order = []
    for c in range(len(cls[-1])):
        order.extend(expand(len(cls) - 1, c))
    return mperm[np.asarray(order, np.int64)]


class Hierarchy:
    """Subdomain and coarsening structure for N vertices and L levels, in
    the Morton order or (``tets`` given, ``order="connectivity"``) the
    connectivity-aware one."""

    def __init__(self, X, levels, tets=None, order="morton", links=None):
        self.N = X.shape[0]
        self.L = levels
        if order == "connectivity":
            self.perm = connectivity_perm(X, tets, levels, links=links)
        elif order == "morton":
            self.perm = morton_perm(X)
        else:
            raise ValueError(order)
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
