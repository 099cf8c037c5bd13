"""Population-annealing Max-Cut engine for one MI355X (arXiv 2510.21105).

Modules:

* ``pa``        -- binding of the C ABI of ``libpa.so`` (``include/pa.h``):
                   ``Solver`` (run, run_steps, checkpoint/restore, results),
                   ``run_batch``, ``build_tables``.
* ``workloads`` -- seeded synthetic graphs, schedules and sweep orders.
* ``gset``      -- G-set files and the cut of a configuration (eq. (1)).
* ``hexcfg``    -- the paper's hexadecimal configuration format (section 3).
* ``serve``     -- serving loop with arrival-order admission under an HBM budget.
* ``solve``     -- command-line solve of a G-set file.
* ``build``     -- in-tree hipcc build of ``libpa.so`` for gfx950.

Every annealing step runs in the library's HIP kernels; there is no CPU path.
"""
