"""Plain, slow, FP64 CPU oracle of the central-moment discrete Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package: only tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP path; the two meet only in
the seeded input generators of ``workloads``, which hold no arithmetic of the
method.

Modules
-------
cdbm      the method itself: discrete velocities (Eqs. (2)-(3)), the moment
          matrix and per-cell equilibrium solve (Eqs. (4)-(7)), macroscopic
          recovery and nonequilibrium measures (Eqs. (8)-(11)), the NND flux
          scheme (Eqs. (12)-(20)), BGK relaxation (Eq. (1)) and the two-stage
          Runge-Kutta step; its adjoint is the reverse-mode derivative of the
          same code (torch.autograd), checked against finite differences.
riemann   exact ideal-gas Riemann solver (for the shock-tube benchmarks).
analytic  Taylor-Green solution (Eqs. (22)-(24)), the Chapman-Enskog estimate
          of Eq. (21), linear acoustic plane waves, Rankine-Hugoniot relations,
          the relative L2 norm of Eq. (25).
"""
