"""Dense product ``y = A v`` with ``A[j,k] = f(x_j, y_k)`` (Sect. 1).  Oracle.

Direct summation in FP64 over all pairs, in row chunks.  ``f`` is zero for
bitwise-coinciding points (the zero diagonal of Sect. 4).
"""
from __future__ import annotations

import numpy as np

from .interpolation import helmholtz


def dense_rows(points_T, points_S, v, kappa, rows, chunk: int = 256) -> np.ndarray:
    X = np.asarray(points_T, dtype=np.float64).reshape(-1, 3)
    Y = np.asarray(points_S, dtype=np.float64).reshape(-1, 3)
    v = np.asarray(v, dtype=np.complex128).reshape(-1)
    rows = np.asarray(rows, dtype=np.int64)
    out = np.zeros(rows.shape[0], dtype=np.complex128)
    for a in range(0, rows.shape[0], chunk):
        x = X[rows[a:a + chunk]]
        d = x[:, None, :] - Y[None, :, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        same = np.all(x[:, None, :] == Y[None, :, :], axis=2)
        r[same] = 0.0
        out[a:a + chunk] = helmholtz(r, kappa) @ v
    return out


def dense_matvec(points_T, points_S, v, kappa, chunk: int = 256) -> np.ndarray:
    n = np.asarray(points_T).reshape(-1, 3).shape[0]
    return dense_rows(points_T, points_S, v, kappa, np.arange(n), chunk)
