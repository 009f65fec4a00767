"""FP64 CPU oracle of the coupled hybrid LB step (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
package.  It shares no code with the HIP path; see core.py for what it
computes and brute.py for the per-site loop version used on tiny boxes.
"""
from . import core, lattice  # noqa: F401
