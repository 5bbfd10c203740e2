"""Plain CSR container used to hand Hamiltonians to the oracle and the GPU path."""

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """Square sparse matrix in compressed-sparse-row form.

    ``row_ptr`` has n+1 int64 entries, ``col`` and ``val`` have nnz entries;
    columns are sorted and unique inside each row.  Values are float64.
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        a[rows, self.col] = self.val
        return a

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def diagonal(self) -> np.ndarray:
        d = np.zeros(self.n)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        m = rows == self.col
        d[rows[m]] = self.val[m]
        return d


def coo_to_csr(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    """Sort (row, col) pairs, sum duplicates, and pack into CSR (int64 indices)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start) if len(vals) else vals
    r = uniq // n
    c = uniq % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return CSR(n, row_ptr, c.astype(np.int64), summed.astype(np.float64))
