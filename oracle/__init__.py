"""FP64 CPU oracle for block-Jacobi PCG map-making -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct reference that the GPU library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import it; the library never does, and the oracle shares no code with the library.

Every function cites the passage of the paper (arXiv:2112.03370) it follows.  Where the paper is
silent the oracle takes a documented reading (listed in the repository's design notes).
"""

from .mapmaking import *  # noqa: F401,F403
from .templates import *  # noqa: F401,F403
from . import mapmaking, templates  # noqa: F401
