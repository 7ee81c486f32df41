"""Worker of the CPU-baseline timing of the oracle (bench.py's cpu_baseline leg).

TEST INFRASTRUCTURE ONLY: it runs the oracle's ladder (eqs. dual_ladder,
lin_alg_inv) on a block of bosonic slices in a worker process, so that the
baseline can time one process and several; it lives here so that worker
processes import it by name.  The product path never imports it.
"""
import time

from . import df_oracle as O


def ladder_seconds(task):
    """task = (gamma^{d/m} [2][k][n][n], chi [k][n][N]): seconds of O.ladder on them."""
    gam, chi = task
    t0 = time.perf_counter()
    O.ladder(gam, chi)
    return time.perf_counter() - t0
