"""CPU FP64 oracle of the CHNS element loop -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
"""
from .oracle import (BLOCK_CH, BLOCK_NS, Mesh, Params, SolverOpts, StepStats,  # noqa: F401
                     build, lib, num_threads, set_num_threads)
