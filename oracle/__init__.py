"""FP64 CPU oracle of the extended lattice Boltzmann step (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package. The product path never calls it.
"""
from .elbm_oracle import *  # noqa: F401,F403
from .elbm_oracle import Params, Diag  # noqa: F401
