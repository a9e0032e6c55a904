"""Reference (oracle) implementation of the separable high-order FEM solve.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow CPU implementation
of what the GPU library computes, written from the paper (Zlotnik & Zlotnik,
"A direct fast FFT-based implementation for high order finite element method
on rectangular parallelepipeds for PDE", arXiv:1609.07758).  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.
The GPU library never imports, links or calls anything here, and nothing here
imports the GPU library: the two share no code.

What it computes, step by step (each module cites the passage it follows):

* ``element``   exact rational local stiffness/mass matrices of the nth-order
                Lagrange element on [-1, 1] (Section 2, paragraph 1) and the
                element eigenproblems of eq. (eig_elem), in mpmath.
* ``assembly``  the global 1D pencil (eq. (eig_glob)) and the N-D operator of
                eq. (bvp glob 2): dense / sparse assembly and a matrix-free
                FP64 apply whose stiffness part is evaluated in difference
                form so that constants stay exactly in its kernel.
* ``spectral``  the 1D eigenpairs of the pencil: (i) a dense FP64
                generalized eigensolve, (ii) a high-precision route that
                solves the n x n Bloch-symbol pencil per wave number in
                mpmath (the paper fixes quadruple precision for the
                eigenvalues, Section 2, paragraph 5) and builds the
                eigenvectors of Theorem 1 (first of the two) from them.
* ``solve``     the plain definition v = (x)V diag(1/(sum 4 h^-2 lam + alpha))
                (x)V^T f^h by dense products along every axis (eq. (decomp v 2)).
* ``load``      the load vector f^h of a given f by (n+1)-point Gauss
                quadrature, and grid coordinates (Section 2, paragraph 5).
* ``varcoef``   the variable-coefficient operator -div(a grad u) + alpha u
                by (n+1)-point Gauss quadrature: assembled, matrix-free, and
                a sparse direct solve.
* ``pcg``       a plain preconditioned CG for the variable-coefficient
                operator (exact constant-coefficient solve as the
                preconditioner); its iteration counts stand beside the GPU's.
* ``timestep``  implicit time stepping (heat: backward Euler; wave: the
                implicit three-level scheme), one solve per step.
* ``periodic``  periodic axes: the assembled periodic pencil and a sparse
                direct solve corrected with exactly evaluated residuals.

Parity status: every function is pinned by a test in ``tests/`` against
values the paper prints, closed forms, invariants or brute force.
"""
