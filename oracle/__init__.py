"""Plain CPU FP64 dense oracle: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may import
or run anything in this package.  The HIP library never calls it and shares no code with it.
"""
from .inla_dense import *  # noqa: F401,F403
