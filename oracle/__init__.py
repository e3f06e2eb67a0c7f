"""FP64 CPU reference of the three-weight message-passing planner.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg.  The product path never imports this package.
"""
from .ref import *  # noqa: F401,F403
