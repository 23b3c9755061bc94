"""Plain FP64 CPU oracle for the PWL current-based volume integral equation.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference against which the GPU library is checked.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the GPU library
(``paper_1902_02196_amd``) and never imports it.

Modules (each function cites the part of the paper it follows; the paper is
Georgakis, Giannakopoulos, Litsarev, Polimeridis, "A Fast Volume Integral
Equation Solver with Linear Basis Functions for the Accurate Computation of EM
Fields in MRI", IEEE TAP 2020):

* ``physics``   - constants and materials (Sec. II, eq. 1-2, 6-7, 17)
* ``toeplitz``  - Galerkin blocks of the N operator for the PWL basis
                  (Sec. III-A/B/C, eq. 19-26, 32-34, 42-43)
* ``unreduced`` - brute-force 6-D quadrature of the dyadic kernel (pin only)
* ``gaussian``  - the same blocks by a second route (power series of g and
                  the Gaussian representation of 1/R, exact 1-D factors), the
                  pin of ``toeplitz`` at touching and coincident voxels
* ``matvec``    - direct voxel-pair sum, preconditioned operator (eq. 16-17,
                  24), circulant FFT product (Sec. IV-A)
* ``incident``  - tested incident fields (eq. 27, 30-31)
* ``solve``     - dense LU and restarted GMRES (Sec. V, GMRES(50))
* ``post``      - fields, absorbed power, error metrics (Sec. IV-C, eq. 44,
                  Sec. V-C error definitions)
* ``magnetic``  - magnetic field h_tot = h_inc + K j with the curl operator
                  K = curl S (eq. 8b, 'tot_fields' b, 25b), b1+, magnetic
                  energy and the errors of Sec. V-D; the K blocks come from
                  ``toeplitz`` (part 'K'), pinned by ``gaussian`` and
                  ``unreduced``
* ``mie``       - Mie series absorbed power for a homogeneous sphere (Sec. V-A),
                  also with a relative permeability (the J-M pin)
* ``jm``        - the J-M formulation with magnetic contrast (Sec. II
                  eq. 13-15): 24 unknowns per voxel, the N and K blocks
                  combined, dense LU for tiny grids, fields and power
* ``tucker``    - Tucker (low multilinear rank) compression of the
                  Toeplitz-defining tensors (Sec. III-C, last paragraph):
                  sequentially truncated HOSVD by SVD of the unfoldings
* ``pwc``       - the piecewise-constant discretisation the paper compares
                  against (Sec. V: 3 unknowns per voxel, 6 unique tensors),
                  as the l = 1 restriction of the PWL system

Parity status: every function is pinned by a ``-m "not gpu"`` test
(closed forms, brute force, invariants, an independent second route, hand-
worked values) except the absolute accuracy of the discretisation against
Mie, which the paper only shows in a figure that is not available ("parity
unpinned" for that trend).
"""
