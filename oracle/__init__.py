"""FP64 CPU oracle for GPU-friendly stroke expansion (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does.
"""
from .oracle import *  # noqa: F401,F403
