"""Every row of the measured launch table (csrc/tuned.inc, written by
paper_2601_17979_amd/tune.py on the GPU) is used by the plan and gives
results within tolerance of the oracle: for each (dtype, n class, tall)
row, a few matrices of a shape inside the class run through the C ABI with
the library's own choices (path BLOCKED, nb and inner solve left open)."""
import os
import re

import numpy as np
import pytest

from workloads import gen
from gpu_util import compare_with_oracle, oracle_batch, run_gpu, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_2601_17979_amd", "csrc", "tuned.inc")
NAMES = {0: ("float32", np.float32), 1: ("float64", np.float64), 2: ("complex64", np.complex64),
         3: ("complex128", np.complex128)}
LOWER = {32: 16, 64: 32, 128: 64, 256: 128, 512: 256}   # class nmax -> the class below


def _rows():
    txt = open(TABLE).read()
    blk = txt[txt.index("kTunedBlock"):txt.index("kTunedResident")]
    rows = []
    for m_ in re.finditer(r"\{\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(-?\d+),", blk):
        rows.append(tuple(int(x) for x in m_.groups()))
    return rows


ROWS = _rows()


@pytest.mark.parametrize("row", ROWS, ids=[f"{NAMES[r[0]][0]}-n{r[1]}-tall{r[2]}" for r in ROWS])
def test_tuned_block_entry(row):
    import torch
    from paper_2601_17979_amd import svdb
    dt, nmax, tall, nb, inner = row
    tname, npdt = NAMES[dt]
    n = LOWER[nmax] + 5                         # inside the class (n <= nmax)
    m = 3 * n if tall else n
    cx = dt in (2, 3)
    plan = svdb.plan(getattr(torch, tname), m, n, path="blocked", precondition=0)
    assert plan[1] == nb, (row, plan)          # the plan takes the table's width
    A = np.stack([gen.family(gen.rng_for(9300 + nmax + tall, k), ("gauss", "geo")[k % 2], m, n,
                             1e6, complex_=cx) for k in range(3)]).astype(npdt)
    say(f"[tuned {tname} {m}x{n}: nb {nb}, inner {inner}]")
    S, U, V, info, sw = run_gpu(A, dtype=getattr(torch, tname), path="blocked", precondition=0)
    wide = np.complex128 if cx else np.float64
    Sr, _, _, _, infor = oracle_batch(A.astype(wide))
    compare_with_oracle(A.astype(wide), S.astype(np.float64), U.astype(wide), V.astype(wide),
                        info, Sr, infor, dtype=npdt, label=f"tuned {tname} {m}x{n}")
