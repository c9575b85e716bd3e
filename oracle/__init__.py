"""FP64 CPU oracle for the Newton-system solve of the arrowhead-LP interior-point
method (Kempke, Rehfeldt, Koch: hierarchical Schur complement approach).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The GPU library never calls it and there is no CPU fallback built on it.

Modules
  lp         constraint operator, norms and the full sparse matrix (Sec. 2.2, 3.2;
             block, link and global rows)
  dense_kkt  brute-force dense solves of the Newton system (Sec. 2.3)
  newton     block elimination: factorization Alg. 2, solve Alg. 3 (Sec. 3.2)
  ipm        Mehrotra predictor-corrector driver (Sec. 2.3; constants are readings)
  bounded    the same driver with upper bounds inside the iteration (slacks and
             duals of their own; Q = W/S in the reduced Newton system)
  sensitivity  derivatives of the mu-fixed KKT map w.r.t. (b, c): forward and
             transposed Newton solves, central-path re-solve for differences

Everything is plain NumPy/SciPy in float64.  Library primitives (matmul,
LAPACK Cholesky, triangular solves) serve as steps; there is no blocking,
fusion or reordering beyond the block elimination the paper states.

Parity status
  newton.factor / newton.solve  pinned: dense LU of the full Newton system,
                                minimum-norm least squares, App. A structure;
                                with global rows in the border (the dense layer
                                of Sec. 4.1): dense LU, the border's inertia
                                (ng, n0), planted mistakes
  ipm.solve                     pinned: known optimum of the generated LP,
                                KKT conditions, scipy's HiGHS on small cases;
                                the iterate trajectory itself is parity unpinned
                                (the paper prints no iterates or counts)
  bounded.solve                 pinned: dense LU of the whole Newton system with
                                bounds, planted mistakes, known optimum with
                                active bounds, HiGHS (also on general forms)
  sensitivity.*                 pinned: dense LU of K', the adjoint identity,
                                central differences of the central-path map,
                                LP closed forms at a nondegenerate optimum
"""
