"""FP64 CPU oracle for the Allen-Cahn Parareal hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import,
call, link or execute anything in this directory; only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it.  It shares
no code with the HIP path: the FFTs here are scipy's, every table is
computed here, and the inputs it is handed come from the seeded input
generators (which hold none of the method's arithmetic).

Modules:
  allen_cahn  -- the fully discrete fine scheme, F, the numerical coarse
                 propagator, Parareal (Algorithm 2), energy / mass / MBP
                 diagnostics and the relative-L2 error metric.

Each function states the passage of the paper (arXiv 2510.07672,
"Parallel-in-Time Solution of Allen-Cahn Equations by Integrating
Operator Learning into the Parareal Method") that it follows.
"""

from .allen_cahn import (  # noqa: F401
    Problem,
    Coarse,
    f_double_well,
    potential,
    laplacian_stencil,
    symbol_mu,
    ssi_step,
    fine,
    coarse_num,
    parareal,
    serial_fine_trajectory,
    discrete_energy,
    mass,
    rel_l2,
)
