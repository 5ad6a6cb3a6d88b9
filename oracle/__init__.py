"""FP64 CPU oracle for the ideal-MHD TVD-MUSCL step (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never does.
"""
from .pyorc import Oracle, OrcConfig, build_oracle, load_oracle  # noqa: F401
