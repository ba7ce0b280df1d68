"""FP64 CPU oracle for the compressed 3D FFL MPI operator and its solvers.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` use it.  It shares
no code with the HIP library (no kernels, headers, helpers or table builders).

The oracle writes out the paper's definitions step by step, in float64:

* ``physics``   -- Langevin function, its derivative, the sinusoidal FFL
                   trajectory and velocity (Sec. 1.2 eq. H0-H1, eq. reals0,
                   Appendix B eq. PSF in its collinear reduction).
* ``geometry``  -- grids, angles and the kept harmonic bins (Sec. 2.1,
                   Appendix A).
* ``projector`` -- the parallel-beam projection P_theta (Sec. 2.2 eq. qtheta,
                   eq. ptheta2, eq. ptheta1) and its exact transpose, plain C
                   loops in ``proj.c``.
* ``signal``    -- the 1D FFL signal model V E H B (eq. stheta1) and the
                   harmonic compression S D_Gamma F (eq. bcompress, eq. DCmodel,
                   Appendix A), plus their real adjoints.
* ``operator``  -- the full block operator A of eq. modelF1 / Sec. 3.3, its
                   adjoint, the operator norm and synthetic data generation.
* ``solvers``   -- CGLS on the Tikhonov objective eq. nummodel, its restart
                   variants, and the paper's momentum gradient method eq. iters.

Parity status of every function is listed in each module header.
"""
