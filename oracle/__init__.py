"""Plain CPU FP64 oracle of the B-char transfer build and apply.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, header,
table or helper with the HIP path in ``paper_1908_05834_amd/``; both sides
receive the same seeded inputs (mesh description, velocity lattice, c) and
compute everything else on their own.

What it computes, per time step (Cheng & Droniou, "An efficient
implementation of mass conserving characteristic-based schemes in 2D and
3D", arXiv:1908.05834):

* ``geometry.ball_layout``        -- balls B_{K,s} and porous density rho_K
                                     (Sec. 3, eq. def:porous.density)
* ``geometry.trace_points``        -- backward tracking of ball centres along
                                     the flow of u/phi (Sec. 2, eq. charac)
* ``geometry.tracked_radius``      -- r_hat = r for constant phi
                                     (eq. ball_volChange), mean distance to
                                     the tracked cardinal points otherwise
                                     (eq. rTrackedBall)
* ``geometry.candidate_pairs``     -- every (tracked ball, residing ball)
                                     pair that overlaps, by brute force or a
                                     k-d tree plus the exact predicate
* ``geometry.disk_lens_area`` /
  ``geometry.sphere_lens_volume``  -- measure of the intersection of two
                                     balls, written as the sum of two
                                     circular segments / spherical caps
* ``transfer.initial_volumes``     -- V (Sec. 3.1, eqs. fracMaterial and
                                     ball_int) as a CSR matrix
* ``transfer.scaling_sweeps``      -- N alternating column/row scalings
                                     (Sec. 3.2, eq. volAdj)
* ``qp.solve_mass_qp``             -- the least-change bounded problem
                                     (Sec. 3.2, eq. opti_masscons)
* ``transfer.apply``, ``transfer.mass`` -- the update (Sec. 2,
                                     eq. phys-inter-ELLAM) and the porous
                                     mass (Sec. 2.1)

Everything is IEEE binary64 with NumPy/SciPy; the only exception is the
FP32-volume mode, where the overlap predicate is evaluated in binary32 on
binary32-rounded centres and radii (NumPy float32 arithmetic, no fused
multiply-add) and the lens is then evaluated in binary64 on those rounded
inputs.

Every function here is pinned by ``tests/test_oracle_*.py`` against
closed forms, special values, Monte Carlo, exact rational arithmetic,
brute force and independent library solvers; see the module docstrings.
"""

from . import geometry, transfer, qp  # noqa: F401
