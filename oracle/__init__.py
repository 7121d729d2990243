"""Plain FP64 CPU oracle of the PeriDEM step -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the CPU-baseline leg of bench.py may import
this package.  It shares no code with the GPU library; both read the same
seeded inputs from paper_2108_07212_amd.workloads.
"""
from .oracle import Oracle, build_oracle, oracle_library_path  # noqa: F401
from .oracle import T_PD, T_SELF, T_NBR, T_WALL, T_BODY, T_ALL  # noqa: F401
from .fragments import components, child_counts  # noqa: F401
