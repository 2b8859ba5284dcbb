"""FP64 CPU oracle of the coupled reactive-transport LB step (test infrastructure).

Only tests/, the package smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path never does.
"""
from .oracle import OracleSim, build_oracle, oracle_lib_path  # noqa: F401
