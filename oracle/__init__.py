"""Plain FP64 CPU oracle for the Crank-Nicolson finite-volume scheme of the
conservative space-fractional diffusion equation and its sine-transform (tau)
preconditioned Krylov solvers (Qu, Lei, Hon, Huang, arXiv 2511.21198).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
execute anything in this package; only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP path: every quantity here is recomputed from the paper's definitions in
plain NumPy/SciPy (float64) or mpmath.

Modules
-------
coeffs     s_k, q_k, eta, A_n and tau eigenvalues            (Section 2, Section 3)
operators  dense assembly (tiny sizes) and structured operators (any size)
krylov     textbook PCG and left-preconditioned restarted GMRES
cn         the Crank-Nicolson time loop
circulant  the comparators of the experiments: no preconditioner, T. Chan's
           and Strang's circulants                           (Section 4)
examples   the manufactured solutions of Examples 4.1 and 4.2 (Section 4)
nn         reference 3D convolution network (forward/backward) for the learned
           warm start

Parity status: every function is pinned by a ``-m "not gpu"`` test against
something other than itself (closed forms, brute force on tiny sizes, the
paper's printed iteration counts, invariants).  Functions without such a pin
say "parity unpinned" in their docstring.
"""
