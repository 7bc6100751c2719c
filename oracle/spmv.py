"""Sparse matrix–vector product from its definition: y_i = Σ_j a_ij x_j.

The CSR row segments (RowPointer, Section 5.3.2) are summed in 80-bit extended
precision (``np.longdouble``, 64-bit significand) so that the reference carries
≈ rowlen·2⁻⁶⁴ relative error instead of the ≈ rowlen·2⁻⁵³ of a plain float64
loop; the comparison then measures the device's error, not the oracle's.
``row_exact`` evaluates one row in exact rational arithmetic and rounds once,
for spot checks at any matrix size.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def spmv(row_pointer, col_index, value, x):
    """y = M x for M in CSR; returned in float64, accumulated in long double."""
    ptr = np.asarray(row_pointer, dtype=np.int64)
    m = len(ptr) - 1
    prod = np.asarray(value, dtype=np.longdouble) * np.asarray(x, dtype=np.longdouble)[np.asarray(col_index)]
    y = np.zeros(m, dtype=np.longdouble)
    nz_rows = np.nonzero(np.diff(ptr))[0]
    if nz_rows.size:
        y[nz_rows] = np.add.reduceat(prod, ptr[nz_rows])
    return y.astype(np.float64)


def spmv_abs(row_pointer, col_index, value, x):
    """(|M| |x|)_i — the natural scale of the rounding error of row i."""
    return spmv(row_pointer, col_index, np.abs(np.asarray(value)), np.abs(np.asarray(x)))


def row_exact(row_pointer, col_index, value, x, i):
    """Row i of M x: exact products and exact sum, rounded once to float64."""
    a, b = int(row_pointer[i]), int(row_pointer[i + 1])
    s = Fraction(0)
    for k in range(a, b):
        s += Fraction(float(value[k])) * Fraction(float(x[col_index[k]]))
    return float(s)
