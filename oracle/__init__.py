"""CPU oracle for the batched one-sided Jacobi SVD.

TEST INFRASTRUCTURE ONLY.  Plain FP64 / complex128 C code (``jacobi_ref.c``)
behind a ctypes front end (``ref.py``).  It shares no code with the GPU
library, and only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may use it.
"""
from .ref import (block_gesvj, block_iter, build, default_tol, gesvj, gesvj_batch,  # noqa: F401
                  heevj, num_threads, precond_gesvj, precond_gesvj_batch, round_robin,
                  row_cyclic, set_num_threads)
