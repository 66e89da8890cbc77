"""FP64 CPU oracle for canonical density-matrix perturbation theory.

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import it; the GPU library and its Python binding never
do.  It shares no code with the GPU path.
"""
from .dmpt_oracle import *  # noqa: F401,F403
from .dmpt_oracle import __all__  # noqa: F401
