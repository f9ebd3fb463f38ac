"""CPU FP64 oracle for the Total Lagrangian internal force (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403
from .constraints import *  # noqa: F401,F403
