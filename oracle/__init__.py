"""CPU oracle of the nested polarized-traces Helmholtz solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, complex128
NumPy/SciPy statement of what the GPU path computes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product path (``paper_1510_01831_amd``) never does.  It shares
no code with the HIP path; the only common module is the seeded input
generator ``paper_1510_01831_amd.media``, which holds no solver arithmetic.

Reference: Zepeda-Nunez & Demanet, "Nested domain decomposition with
polarized traces for the 2D Helmholtz equation" (arXiv 1510.01831).

Modules
  discretization -- App. A: extended grid, quadratic PML, 5-point operator
                    (symmetric row scaling), layer and cell windows.
  polarized      -- Sec. 2.2-3 and 4.1: Green's integrals from App. C's
                    equivalent sources, the SIE, the polarized system, the
                    Gauss-Seidel sweeps, reconstruction (Alg. 6).
  nested         -- Sec. 4.2: cells, inner SIE, block LU without pivoting
                    (Sec. 4.2.2), volume solve (Alg. 7) and the interface
                    factorisation (eq. factorization).
  nested_pt      -- Sec. 4.2.1: nested polarized traces, the inner SIE as a
                    polarized system over the cells, iterated by GMRES with
                    the inner Gauss-Seidel sweeps.
  gmres          -- left-preconditioned GMRES (the Krylov driver of Alg. 6).
  forms          -- mixed-precision refinement and the adjoint-state
                    gradient of a least-squares misfit.

Every function that has no independent pin says "parity unpinned" in its
docstring.
"""
