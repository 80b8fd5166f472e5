"""FP64 CPU oracle for DCF-PCA. TEST INFRASTRUCTURE: only the test suite,
the smoke check and the benchmark's CPU-baseline leg use it."""
from .reference import *  # noqa: F401,F403
from .reference import __all__  # noqa: F401
