"""Contact classification, localized Top-K and the updated fine blocks (FP64).

Test infrastructure (see the package docstring).

Section 4.1.1 (construction of the local update matrices):
* every current contact is compared with its state in the base set taken
  at the last restart, using its identity key;
* not in the base set (new): u = sqrt(k) n, dS = k;
* in the base set with a rotated normal: treated as new, the base stiffness
  stays in H_base; the paper compares n_curr . n_base with an angle
  threshold; this oracle reads it as cos(angle(n_curr, n_base)) < cos(eps_rot)
  on the full stencil vector n = grad d, eps_rot = 25 degrees;
* stable normal and stiffer (k > k_base): u = sqrt(k - k_base) n_curr,
  dS = k - k_base;
* stable normal and not stiffer: ignored (dS = 0).  Base contacts that are
  no longer current are ignored as well (they stay in H_base).
* per subdomain, the candidates (contacts whose stencil has a vertex in it)
  are ranked by dS, descending, ties by key ascending, and the first K form
  U_d, whose columns are S_d u.

The global U used for the curvature model H~ = H_base + U U^T (Section 4.1,
Eq. for H~; supplement Eq. (11)) holds every contact with dS > 0, untruncated.

Section 4.1.2: the updated block is (S_d H_base S_d^T + U_d U_d^T)^-1; the
oracle forms that matrix and inverts it directly, the plain definition the
Woodbury formula reaches.
"""
from __future__ import annotations

import numpy as np

from . import fem
from .mas import SUB

NONE, NEW, ROTATED, STIFFEN, SOFTEN = 0, 1, 2, 3, 4


def classify(problem, base, curr, cos_rot=np.cos(np.deg2rad(25.0))):
    """Returns (dS (m,), u (m,12), case (m,)) for the current contacts."""
    k_cur = problem.contact_stiffness(curr['d'])
    k_base = problem.contact_stiffness(base['d'])
    where = {int(k): i for i, k in enumerate(base['key'])}
    m = curr['key'].shape[0]
    dS = np.zeros(m)
    u = np.zeros((m, 12))
    case = np.zeros(m, np.int32)
    for c in range(m):
        n = curr['grad'][c]
        k = k_cur[c]
        b = where.get(int(curr['key'][c]))
        if b is None:
            case[c] = NEW
            s = k
        else:
            nb = base['grad'][b]
            cosang = float(n @ nb) / (np.linalg.norm(n) * np.linalg.norm(nb))
            if cosang < cos_rot:
                case[c] = ROTATED
                s = k
            elif k > k_base[b]:
                case[c] = STIFFEN
                s = k - k_base[b]
            else:
                case[c] = SOFTEN
                s = 0.0
        if s > 0:
            dS[c] = s
            u[c] = np.sqrt(s) * n
    return dS, u, case


def topk(hier, curr, dS, u, K):
    """dict: subdomain -> list of contact indices (ranked), at most K."""
    cand = {}
    for c in np.nonzero(dS > 0)[0]:
        seen = set()
        for j in range(4):
            v = curr['idx'][c, j]
            if v < 0:
                continue
            d = int(hier.subdomain_of_vertex(v))
            if d in seen:
                continue
            # S_d u must be nonzero
            nz = False
            for jj in range(4):
                vv = curr['idx'][c, jj]
                if vv >= 0 and hier.subdomain_of_vertex(vv) == d and np.any(u[c, 3 * jj:3 * jj + 3] != 0):
                    nz = True
            if nz:
                seen.add(d)
                cand.setdefault(d, []).append(c)
    out = {}
    for d, lst in cand.items():
        lst = sorted(lst, key=lambda c: (-dS[c], int(curr['key'][c])))
        out[d] = lst[:K]
    return out


def local_U(hier, curr, u, d, cols):
    """Dense S_d U_d (3 n_d x r) for the selected contacts of subdomain d."""
    dofs = hier.subdomain_dofs(d)
    pos = {int(q): i for i, q in enumerate(dofs)}
    Ud = np.zeros((dofs.size, len(cols)))
    for j, c in enumerate(cols):
        for jj in range(4):
            v = curr['idx'][c, jj]
            if v < 0:
                continue
            for a in range(3):
                i = pos.get(int(3 * v + a))
                if i is not None:
                    Ud[i, j] += u[c, 3 * jj + a]
    return Ud


def updated_blocks(hier, H_base, curr, u, sel):
    """Level-0 inverses of S_d H_base S_d^T + U_d U_d^T for every d."""
    blocks = []
    for d in range(hier.num_subdomains(0)):
        dofs = hier.subdomain_dofs(d)
        M = H_base[dofs][:, dofs].toarray()
        if d in sel:
            Ud = local_U(hier, curr, u, d, sel[d])
            M = M + Ud @ Ud.T
        blocks.append(np.linalg.inv(M))
    return blocks


def global_U(problem, curr, u, dS):
    """Sparse U with one column per contact with dS > 0 (untruncated)."""
    keep = dS > 0
    return fem.update_matrix(curr['idx'][keep], u[keep], problem.N)
