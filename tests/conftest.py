import ctypes
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The FP64 oracle allocates large temporaries per object; with glibc's defaults each is a fresh
# mmap that is returned on free, so every call pays its page faults again (about 25x the
# arithmetic at the stress workload's sizes). Keep large blocks on the heap and freed memory in
# the process. An allocator setting only: the oracle's code and arithmetic are unchanged.
try:
    _libc = ctypes.CDLL("libc.so.6")
    _libc.mallopt(-3, 1 << 30)   # M_MMAP_THRESHOLD
    _libc.mallopt(-1, 1 << 34)   # M_TRIM_THRESHOLD
except OSError:
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
