"""Low-rank coupling matrices by adaptive cross approximation (Sect. 2.7).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper compresses each coupling matrix as A ~ U V^* with partially
pivoted ACA and leaves the rank to a tolerance.  Written here from the
method's definition: cross k takes the residual of one row of A (the pivot
row), normalises it by its largest entry (the pivot column), takes the
residual of that column, and moves to the row where the new column is
largest among the rows not used yet.  Only the pivot rows and columns of A
are evaluated.  The loop stops when the new cross is small against the
approximation built so far, ||u_k|| ||v_k|| <= eps ||S_k||_F, with the
Frobenius norm of S_k = sum_l u_l v_l^T updated from inner products (no
matrix is formed).

Pinned by: exact recovery of matrices of known rank (with zero rows), the
error of the Helmholtz coupling matrices against the tolerance and against
the SVD's best error at the same rank, and the matvec with compressed
couplings against the dense-coupling matvec.
"""
from __future__ import annotations

import numpy as np


def aca(row, col, n_rows: int, n_cols: int, eps: float, max_rank: int | None = None):
    """Partially pivoted ACA of the n_rows x n_cols complex matrix whose rows
    and columns ``row(i)`` / ``col(j)`` return.  Returns (U, W) with
    A ~ U @ W.conj().T, U (n_rows, k), W (n_cols, k)."""
    max_rank = min(n_rows, n_cols) if max_rank is None else max_rank
    us: list[np.ndarray] = []
    vs: list[np.ndarray] = []  # A ~ sum_l u_l v_l^T
    used = np.zeros(n_rows, dtype=bool)
    norm2 = 0.0
    i = 0
    while len(us) < max_rank:
        r = np.array(row(i), dtype=np.complex128)
        for u, v in zip(us, vs):
            r -= u[i] * v
        used[i] = True
        j = int(np.argmax(np.abs(r)))
        if r[j] == 0:  # residual row vanishes: try a row not used yet
            free = np.flatnonzero(~used)
            if free.size == 0:
                break
            i = int(free[0])
            continue
        v = r / r[j]
        u = np.array(col(j), dtype=np.complex128)
        for ul, vl in zip(us, vs):
            u -= vl[j] * ul
        cross = sum((np.vdot(ul, u) * np.vdot(vl, v)).real for ul, vl in zip(us, vs))
        nu, nv = np.linalg.norm(u), np.linalg.norm(v)
        norm2 += 2.0 * cross + (nu * nv) ** 2
        us.append(u)
        vs.append(v)
        if nu * nv <= eps * np.sqrt(max(norm2, 0.0)):
            break
        a = np.abs(u)
        a[used] = -1.0
        if a.max() < 0:
            break
        i = int(np.argmax(a))
    if not us:
        return np.zeros((n_rows, 0), np.complex128), np.zeros((n_cols, 0), np.complex128)
    U = np.stack(us, axis=1)
    W = np.conj(np.stack(vs, axis=1))
    return U, W


def aca_dense(A: np.ndarray, eps: float, max_rank: int | None = None):
    """ACA of an explicit matrix (rows and columns read from it)."""
    A = np.asarray(A)
    return aca(lambda i: A[i, :], lambda j: A[:, j], A.shape[0], A.shape[1], eps, max_rank)
