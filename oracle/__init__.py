"""FP64 CPU oracle of the HEEPS/MARE facet-sum path.

TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package.  The product path never
does, and this package imports nothing from the product.
"""
from .oracle import *  # noqa: F401,F403
