"""FP64 CPU oracle for the CNT-GW hot path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path never does.
"""
from . import gw_oracle  # noqa: F401
