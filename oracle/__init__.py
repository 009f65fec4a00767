"""FP64 CPU oracle of the coupled hybrid LB step (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
package.  It shares no code with the HIP path; see core.py for what it
computes, brute.py for the per-site loop version used on tiny boxes and
d3q15.py for the paper's own LB scheme (D3Q15, stress in the equilibrium) and
pc4.py for its integrator of the order parameters (predictor-corrector,
first-order upwind, fourth-order stencils).
"""
from . import core, d3q15, lattice, pc4  # noqa: F401
