"""Plain FP64 CPU oracle for the staggered space-time DG pressure path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_1601_07384_amd``) and never imports it.

It follows Tavelli & Dumbser, "A staggered space-time discontinuous Galerkin
method for the three-dimensional incompressible Navier-Stokes equations on
unstructured tetrahedral meshes" (arXiv 1601.07384):

* quadrature.py  - simplex rules (Grundmann-Moeller), Gauss-Legendre time
                   rule, and the collapsed face rule used for the Rusanov flux.
* basis.py       - nodal Lagrange basis (Sec. 2.3, eq. bf_1), Taylor modal
                   dual basis (eq. bf_2), Gauss-Legendre Lagrange time basis.
* mesh.py        - primary mesh, faces, left/right elements, dual elements
                   (Sec. 2.2.1).
* spacetime.py   - the literal space-time matrices of Sec. 2.4-2.5 (MD_2..MD_6,
                   vis3, vis11, mj) integrated with space-time quadrature.
* pressure.py    - the pressure Schur operator (eq. CS_19), its assembly, the
                   anchored solve.
* picard.py      - the Picard pressure-correction step (Sec. 2.6, steps 0-6).
* mlp.py         - the multilayer perceptron used as a Krylov initial guess.

Matrices are evaluated in numpy.longdouble (x87 80-bit) and results returned
as float64: the dual mass matrices of the Taylor basis are ill-conditioned at
high degree (condition numbers near 1e10 at p = 4).  Nothing here is blocked,
fused or reordered beyond what the paper's definitions state.
"""
