"""FP64 CPU oracle for the DIA kernel fit — test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use it;
the GPU library never imports, links or calls anything here.
"""
from .oracle import *  # noqa: F401,F403
from .oracle import build_oracle  # noqa: F401
