"""FP64 CPU oracle for the implicit FE step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library and its Python binding
never import it, and it imports nothing from them; the two sides share only the
seeded input generators in ``synth``.

What it computes (paper: Zeng & Courtecuisse, "Efficient parallelization
strategy for real-time FE simulations", arXiv 2306.05893):

* elements.py  -- per-element internal force f_e, tangent stiffness K_e and
                  consistent mass M_e for TET4 / HEX8 with neo-Hookean or
                  St Venant-Kirchhoff material (textbook formulas; the paper
                  names its materials in Sec. 3.1 but prints no formulas).
* assembly.py  -- the triplet list in fill order, the CSR pattern and the
                  triplet -> CSR map built by a plain comparison sort (Sec. 4.2,
                  Table "build pattern"), with the projective Dirichlet rule of
                  Sec. 6.1 (fixed rows/cols dropped, 1 on the diagonal).
* step.py      -- the linear system A a = b of Eq. "dynamic equation2" with
                  A = (1 + h alpha) M + h (beta + h) K and the right-hand side
                  derived from the Taylor expansion of Sec. 3.2 (reading R1),
                  solved directly, then the backward-Euler update of
                  Eq. "implicit integration".
* solve.py     -- dense Cholesky, banded Cholesky and FP64 Jacobi-PCG solves;
                  any x whose relative residual meets the tolerance is a
                  correct solve, the preconditioner only changes speed (Sec. 3.3).
* adjoint.py   -- reverse-mode recursion of the step (not in the paper), with
                  the third-derivative term by complex step, and a complex-step
                  derivative of the whole rollout used to pin it.
* contact.py   -- contact through Lagrange multipliers (Sec. 6.2): the
                  compliance matrix W = H A^{-1} H^T by one solve with many
                  right-hand sides, projected Gauss-Seidel on its
                  complementarity problem, and the motion correction.

Every function is plain and unblocked; vectorisation runs over elements only.
"""
