"""Which storage the SpMV plan picks for a CSR matrix (mirrors the rule in
the library so that tests can state which kernel they exercise)."""
import numpy as np


def dia_ndiag(A):
    """Diagonals of the storage the plan picks (automatic plan): the number of
    distinct column offsets col - row when it is at most 32 and 8 bytes per
    diagonal and row is at most 85% of CSR's 12 per entry + 4 per row, else
    0 (CSR)."""
    if A.n == 0 or A.nnz == 0:
        return 0
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    nd = np.unique(A.col - rows).size
    limit = min(32, (85 * (12 * A.nnz + 4 * (A.n + 1))) // (100 * 8 * A.n))
    return nd if nd <= limit else 0
