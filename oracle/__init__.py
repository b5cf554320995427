"""Plain FP64 CPU oracle for the MAS-PNCG hot path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the HIP library is checked against.  Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import it; the library never calls it and shares no code with it.

Everything is float64 and follows the paper's definitions directly:

* ``fem``       incremental potential (Eq. for E(x) in Section 3.1): inertia,
                stable Neo-Hookean elasticity, log barrier; gradient; the
                SPD-projected Hessian snapshot assembled as a sparse matrix
                (Section 4.1, projected contact Hessian k n n^T).
* ``mas``       Morton subdomains and the multilevel additive Schwarz
                preconditioner, every block formed from the assembled matrix
                and inverted densely (Section 3.3; supplement Section 1).
* ``woodbury``  contact classification and localized Top-K (Section 4.1.1);
                the updated fine blocks by direct dense inversion of
                S_d (H_base + U_d U_d^T) S_d^T (the plain definition behind
                the localized Woodbury solver of Section 4.1.2).
* ``pncg``      2x2 subspace step with fallback (Section 4.2; supplement
                Section 2), restart ratio (Section 4.3), the affine safe step
                and the PNCG loop of Algorithm 1.

Vectors are flat (3N,) arrays in the caller's original vertex order with
xyz interleaved.  Contact sets are dicts with ``key`` (uint64), ``idx``
(m,4) int32 padded with -1, ``grad`` (m,12) = dd/dx, and ``d`` (m,).
"""
