"""FP64 CPU oracle of the EEG lead-field build (test infrastructure only).

This package is the correctness reference for the HIP library.  It is plain,
slow and written to be checked against the paper by eye:

* ``fem``       -- stiffness matrix, complete-electrode-model terms, ground
                   fix and preconditioner diagonal (App. A.1, matrices A, B, C
                   of Eq. (u_system));
* ``source``    -- the source matrix G for point dipoles (App. A.1, entries
                   g_ij; the partial-integration reading of Sec. 2 "Primary
                   current model");
* ``solve``     -- transfer matrix T = A^-1 B (App. A.4) by a direct
                   factorisation, and the preconditioned conjugate gradient of
                   Sec. 2.3.1 one column at a time;
* ``leadfield`` -- the EEG lead field of App. A.2, Eq. (aku), and the
                   reciprocity check that solves the full block system;
* ``sphere``    -- the closed-form multilayer-sphere dipole potential used to
                   pin the oracle against physics;
* ``eit``       -- the linearized EIT lead field of App. A.3;
* ``gnn``       -- the mesh-graph network of the learned PCG warm start
                   (forward, backward, Adam), the reference for its kernels.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  The product library never calls it, and it shares
no code with the HIP path: its inputs are plain numpy arrays produced by the
seeded generators.

Parity status of each function is stated in its docstring; every function is
pinned by a ``-m "not gpu"`` test in ``tests/test_oracle_*.py``.
"""

from . import fem, source, solve, leadfield, sphere, eit, gnn  # noqa: F401
