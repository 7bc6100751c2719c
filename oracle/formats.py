"""Sparse storage formats, written out from their definitions (Section 5.3).

COO (5.3.1): Value, RowIndex, ColumnIndex, sorted by row then column.
CSR (5.3.2): RowIndex compressed into RowPointer = [0, cumsum(row counts)],
             so RowPointer[m] = nnz.
CSC (5.3.3): the column-major twin; CSC of A is read as CSR of Aᵀ by swapping
             m↔n and ColumnPointer↔RowPointer.
Upper-triangle → full symmetric P (Section 6.2): the library stores full P.
"""
from __future__ import annotations

import numpy as np


def dense_to_coo(M):
    """Row-major scan of a dense matrix: the unique sorted COO triplet."""
    M = np.asarray(M, dtype=np.float64)
    r, c = np.nonzero(M)
    return M[r, c].copy(), r.astype(np.int64), c.astype(np.int64)


def coo_to_csr(value, row_index, col_index, m):
    """Compress RowIndex: count per row, then exclusive cumulative sum with a leading 0."""
    order = np.lexsort((col_index, row_index))
    counts = np.zeros(m, dtype=np.int64)
    for r in row_index:
        counts[r] += 1
    row_pointer = np.zeros(m + 1, dtype=np.int64)
    for i in range(m):
        row_pointer[i + 1] = row_pointer[i] + counts[i]
    return np.asarray(value)[order], row_pointer, np.asarray(col_index)[order]


def coo_to_csc(value, row_index, col_index, n):
    """CSC = CSR of the transpose: swap the roles of rows and columns."""
    v, cp, ri = coo_to_csr(value, col_index, row_index, n)
    return v, ri, cp


def csr_transpose(row_pointer, col_index, value, ncols):
    """CSR of Mᵀ from CSR of M (equivalently, CSC of M), by a counting pass."""
    m = len(row_pointer) - 1
    counts = np.bincount(np.asarray(col_index, dtype=np.int64), minlength=ncols)
    t_ptr = np.zeros(ncols + 1, dtype=np.int64)
    t_ptr[1:] = np.cumsum(counts)
    rows = np.repeat(np.arange(m), np.diff(row_pointer))
    # stable placement by column: rows are visited in increasing order, so each
    # transposed row's column indices come out sorted
    order = np.argsort(col_index, kind="stable")
    return t_ptr, rows[order], np.asarray(value, dtype=np.float64)[order]


def triu_to_full(colptr, rowidx, val, n):
    """Full symmetric P (CSR) from the upper triangle of P given in CSC.

    Entry (i, j) with i ≤ j of the triangle gives P_ij and, if i ≠ j, P_ji.
    Returns (row_pointer, col_index, value) of full P with sorted columns.
    """
    cols = np.repeat(np.arange(n), np.diff(colptr))
    rows = np.asarray(rowidx, dtype=np.int64)
    v = np.asarray(val, dtype=np.float64)
    if np.any(rows > cols):
        raise ValueError("entry below the diagonal in an upper-triangular input")
    off = rows != cols
    R = np.concatenate([rows, cols[off]])
    C = np.concatenate([cols, rows[off]])
    V = np.concatenate([v, v[off]])
    order = np.lexsort((C, R))
    R, C, V = R[order], C[order], V[order]
    ptr = np.zeros(n + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(np.bincount(R, minlength=n))
    return ptr, C, V
