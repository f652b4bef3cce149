"""Plain, slow, FP64 CPU oracle for periodic Coulomb sums and charge equilibration.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it. It shares no code with the HIP library.

Contents (each function cites the passage of the paper it follows):

* ``ewald``  -- direct Ewald: brute-force real-space erfc sum over every pair
                and periodic image, plain reciprocal k-sum, self and
                neutralising-background terms (Section "Regular Ewald
                Summation", equations ewald_general, ewald_real, ewald_rec,
                ewald_self).
* ``spme``   -- smooth particle-mesh Ewald in FP64 (Algorithm "Smooth PME",
                steps 1-5), written as the plain definition with numpy FFTs.
* ``pairs``  -- the canonical neighbour pair set by brute force (Section
                "Cell based Neighbor List"; the cell method must reproduce it).
* ``qeq``    -- dense Coulomb matrix, bordered QEQ solve (equation
                linear_qeq), matrix-free product (the Cv identity), shadow
                charges q[n] (equation diag_linear_qeq), the Jacobian J and a
                plain GMRES(m) iterate for J x = -(q[n]-n) (equation Jnddot).
* ``grad``   -- gradients of the QEQ energy and vector-Jacobian products
                through the QEQ solve, plus central finite differences.

Units: Angstrom, elementary charge, eV; the Coulomb constant is
``KE = 14.3996454784`` eV*A/e^2.

Parity status: every function is pinned by the CPU tests in ``tests/``
(closed forms, lattice constants, invariances, brute force, library routines).
"""
from .ewald import KE, wrap, real_space, reciprocal_direct, self_background, ewald_direct  # noqa: F401
from .spme import bspline, bspline_deriv, spme_reciprocal, spme_full  # noqa: F401
from .pairs import neighbor_pairs  # noqa: F401
from . import qeq, grad  # noqa: F401
