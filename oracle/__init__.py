"""FP64 CPU oracle of the Shan-Chen bubble growth / merging step (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg import this package.
The product library neither links nor calls it.
"""
from .oracle import OracleSim, label_mask, feq, lattice, uniform, splitmix64, num_threads  # noqa: F401
