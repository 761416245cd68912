"""FP64 CPU oracle of the tree-based column-density method (test
infrastructure only: the tests, the smoke check and the CPU-baseline leg of
the benchmark use it; the product path never does)."""
from .oracle import *  # noqa: F401,F403
