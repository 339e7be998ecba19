"""FP64 CPU oracle for the randomized block Krylov truncated T-SVD.

Test infrastructure only (tests/, __graft_entry__.smoke(), bench.py's
cpu_baseline leg).  It shares no code with the HIP library.
"""
from .tsvd_oracle import *  # noqa: F401,F403
from . import tsvd_oracle  # noqa: F401
