"""CPU FP64 oracle of the KFBI time-stepping method (Tan, Huang, Ying,
"A GPU-accelerated Cartesian grid method for the heat, wave and Schroedinger
equations on irregular domains").

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the
graft entry point and the CPU-baseline leg of the benchmark may import or run
anything in this package.  The product path (the HIP library and its Python
binding) never routes through it, and the two share no code.

The oracle is deliberately plain: numpy/scipy in float64 / complex128, each
function following the paper's section or equation it names, with no
blocking, fusion or reordering beyond the definitions.  Where the paper is
silent or garbled the oracle takes a documented reading (numbered R1..R24 in
the design notes) and says so where it is used.

Modules
    geometry   curve, collocation points, node classes, crossings, stencils
    boxsolve   the five-point (Delta_h - kappa) solve on the box, u = 0 on dB
    interface  jumps, corrections, extraction: one interface-problem solve
    gmres      restarted GMRES with modified Gram-Schmidt
    bie        the Dirichlet boundary integral equation and its solution
    steppers   heat (Crank-Nicolson), wave (theta-scheme), Schroedinger
               (Strang splitting) time steps
    norms      error norms of the numerical examples

Parity status: every module is pinned by tests under tests/ (test_oracle_*),
except the Schroedinger stepper on the wave-packet workload, whose absolute
values have no closed form ("parity unpinned" for that workload; the stepper
itself is pinned by the V = 0 closed-form solution and by convergence order).
"""
