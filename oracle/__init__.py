"""CPU oracle for the tensor-product nth-order FEM Poisson solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code, tables or constants with the GPU
path.

It computes the plain definitions, slowly and in float64 (exact rationals or
mpmath where noted):

* ``element``  -- reference-element stiffness/mass matrices, exactly (Sect. 2).
* ``fem1d``    -- the global 1D scaled operators and their dense generalized
                  eigendecomposition (Sect. 2, the pencil A v = lambda C v).
* ``eigen1d``  -- the eigenpairs in the paper's own form (Sect. 3, Theorem 1:
                  roots of the secular equation, the vectors p_k, s_k).
* ``transforms`` -- direct FC_n and inverse F_n transforms by their
                  definitions (Sect. 3, Theorem 2), O(K^2) sums.
* ``solve``    -- the N-D operator of Sect. 4 and u = A^{-1} f by dense
                  per-axis eigendecomposition plus float64 refinement, and by
                  dense Cholesky for tiny meshes.
* ``loads``    -- Gauss-quadrature load vectors and errors for manufactured
                  solutions (Sect. 5).

Parity status: every public function is pinned by a ``-m "not gpu"`` test
against values printed in the paper, closed forms, textbook special cases or
brute force; see tests/test_oracle_*.py.
"""
