"""FP64 CPU oracle of the ghost-cell IBM projection.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
CPU-baseline leg of ``bench.py``.  It shares no code with the HIP library.
"""
from .oracle import OracleProblem, OracleOpts, build_oracle, lib_path  # noqa: F401
