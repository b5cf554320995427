"""3x3 block-Jacobi preconditioner (FP64): the comparison preconditioner
of the paper's preconditioner-efficacy study (Section 5).

Test infrastructure (see the package docstring).  For a symmetric matrix H
on 3N DOFs (xyz interleaved per vertex), P = blockdiag(H_ii)^-1 with H_ii
the 3x3 diagonal block of vertex i, inverted densely.  In the PNCG loop H
is H~ = H_base (+ U U^T), the same Hessian model that the MAS
preconditioner and the subspace step see.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def vertex_blocks(H):
    """(N, 3, 3) diagonal blocks of a 3N x 3N matrix (sparse or dense)."""
    H = sp.csr_matrix(H)
    n = H.shape[0] // 3
    out = np.zeros((n, 3, 3))
    for a in range(3):
        for b in range(3):
            out[:, a, b] = H[3 * np.arange(n) + a, 3 * np.arange(n) + b].A1
    return out


def inverse_blocks(H):
    """The block-Jacobi inverse as (N, 3, 3) dense inverses."""
    return np.linalg.inv(vertex_blocks(H))


def apply(inv, g):
    """z_i = B_i^-1 g_i."""
    return np.einsum('nab,nb->na', inv, np.asarray(g, np.float64).reshape(-1, 3)).reshape(-1)
