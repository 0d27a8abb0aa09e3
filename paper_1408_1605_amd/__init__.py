"""MI355X-native (gfx950) single-GPU breadth-first search.

The search runs in hand-written HIP kernels inside libbfsmi.so, behind the C
ABI declared in include/bfs.h.  This package only holds that library's
sources (csrc/), its build script and a thin ctypes binding whose functions
carry the C names.
"""
from .binding import *  # noqa: F401,F403
from .binding import Graph, BFSError, bfs_stats, load, LIB_PATH, EXPORTS  # noqa: F401
