"""CPU FP64 oracle of the vLBM update (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never does.
"""
from .oracle import *  # noqa: F401,F403
