"""Plain, slow FP64 CPU oracle for the range-separated (RS) tensor pose scorer.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports, calls or
links it, and this package never imports the product path: the two share only
the seeded input generators in ``workloads/``.

Source: Benner, Khoromskij, Khoromskaia, Stein, "Fast tensor-based electrostatic
energy calculations in the perspective of protein-ligand docking problem"
(arXiv 2510.26611).  Each function cites the passage it follows.

Modules
    sinc    -- Gaussian-sum (sinc quadrature) approximation of 1/r, eq. 2.2
    tensor  -- grid, 1-D Gaussian factor columns, uncompressed long-range tensor, eqs. 2.1-2.6
    rhosvd  -- canonical -> Tucker (RHOSVD) -> canonical rank reduction, Algorithm TEP step 4
    score   -- pose transform, long/short-range potential, energy, vdW flag, gradients
               (Sec. 3.2 Lemma 3.3 / eq. 3.10, Algorithm PLIE, eq. 3.14, eqs. 3.12 and 5.2-5.3)
    direct  -- direct Coulomb binding energy and forces, eq. 3.5 and the force formula of Sec. 3.3
    constants -- derivation of the frozen quadrature step and short-range cutoff

Parity status: every function is pinned by a test in ``tests/test_oracle_*.py``
against closed forms, textbook/library routines, invariants or brute force.
"""
