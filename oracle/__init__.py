"""CPU oracle for the matrix-free DG hot path (test infrastructure only).

This package is a plain, slow, fp64 NumPy/SciPy restatement of the
discretisation in Krank, Fehn, Wall & Kronbichler, "A high-order
semi-explicit discontinuous Galerkin solver for 3D incompressible flow with
application to DNS and LES of turbulent channel flow" (arXiv:1607.01323).
It assembles element and face matrices by direct quadrature (no sum
factorisation) and runs textbook Krylov/Chebyshev/Lanczos iterations.

It is TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_1607_01323_amd``) never imports, links or executes anything here, and
this package never imports the product.  The two share no code; only the
seeded input generators in ``dgmf_inputs`` (which hold no arithmetic of the
method) serve both.

Modules
-------
basis       1D nodal Gauss-Lobatto Lagrange basis and Gauss rule (Sec. 3.1, Sec. 5)
mesh        axis-aligned box meshes, periodic / Dirichlet / Neumann faces, tanh grading
            (Sec. 3.1 tessellation; Sec. 7.1 hyperbolic channel mesh mapping)
sipg        SIPG Laplace / Helmholtz element and face matrices, penalty
            (Sec. 3.2 eqs. poissonspat, ipflux, taue, tau and the viscous step;
            Sec. 4.4 matrix form)
curved      SIPG operator on iso-parametric curved cells: the degree-k interpolant
            of a smooth periodic deformation of the box, point-by-point
            quadrature (Sec. 5, curved cells)
kron        Kronecker-sum construction and fast-diagonalisation direct solve
            on uniform Cartesian meshes (a second, independent construction)
solvers     textbook PCG, Lanczos, Chebyshev (Sec. 5.1 "Solving linear systems")
convective  divergence-form convective operator with local Lax-Friedrichs
            flux, its JVP/VJP and assembled Jacobian (Sec. 3.2 eq. convstepspat)
rng         SplitMix64 counter-based generator (published definition)
multigrid   geometric multigrid V-cycle preconditioner (Sec. 5.1, Poisson solver)
v3          divergence and gradient operators, mass, div-div penalty and the
            local projection of variant V3c (eqs. av3, bv3, div-div, tauD, project)
viscous     the viscous operator in the symmetric-gradient form (SIPG, Sec. 3.2)
mass        block-diagonal inverse mass matrix and the explicit convective
            substep of the matrix form (eq. advect)

Every function that has no independent pin says so; see the test-suite
docstrings for the pins (closed forms, invariants, brute force).
"""
