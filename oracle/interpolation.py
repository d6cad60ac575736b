"""Directional tensor Chebyshev interpolation (Sect. 2.2, 2.5, 2.7).  Oracle.

* Kernel (Sect. 1): ``f(x,y) = exp(i kappa |x-y|) / (4 pi |x-y|)``; reading
  for coinciding points: ``f(x,x) = 0`` (Sect. 4 zeroes the diagonal; here
  ``f`` is zero exactly when the two points are bitwise equal).
* ``f_c(x,y) = f(x,y) exp(-i kappa <x-y, c>)`` (Sect. 2.2).
* Chebyshev nodes of order ``m+1`` on ``[a,b]``:
  ``(a+b)/2 + (b-a)/2 * x_nu``.  Reading: the printed node formula has its
  ``pi`` in the denominator, which would crowd all nodes into [0.959, 1];
  the standard first-kind nodes ``x_nu = cos((2 nu - 1) pi / (2 (m+1)))``,
  ``nu = 1..m+1``, are used.
* Multi-index order (the paper's "suitably ordered"): ``j = (nu1-1)(m+1)^2 +
  (nu2-1)(m+1) + (nu3-1)``, first axis slowest.
* Coupling matrix (Sect. 2.2): ``A_{c,t x s}[j,k] = f_c(xi_{t,alpha_j},
  xi_{s,beta_k})``; it depends only on the level and the offset of the two
  boxes (Sect. 2.7), so it is evaluated once per (level, offset) from the
  node differences ``xi_t - xi_s = (m_t - m_s) + (xi_t - m_t) - (xi_s - m_s)``.
* Transfer matrix (Sect. 2.5, 2.7): ``E_{t',c} = E^d_{t',c} E_{t'}`` with
  ``E_{t'}[j,k] = L_{t,nu_k}(xi_{t',nu_j})`` (one of 8 reference matrices)
  and ``E^d = diag(exp(i kappa <xi_{t',nu}, c - c'>))``.
"""
from __future__ import annotations

import numpy as np


def helmholtz(r: np.ndarray, kappa: float) -> np.ndarray:
    """``exp(i kappa r) / (4 pi r)``, with 0 where ``r == 0``."""
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros(r.shape, dtype=np.complex128)
    nz = r != 0
    rr = r[nz]
    out[nz] = np.exp(1j * kappa * rr) / (4.0 * np.pi * rr)
    return out


def chebyshev_nodes(m: int) -> np.ndarray:
    nu = np.arange(1, m + 2)
    return np.cos((2 * nu - 1) * np.pi / (2 * (m + 1)))


def lagrange_1d(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Lagrange basis of ``nodes`` evaluated at ``x``: shape (len(x), n)."""
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    n = nodes.shape[0]
    out = np.ones((x.shape[0], n))
    for nu in range(n):
        for mu in range(n):
            if mu != nu:
                out[:, nu] *= (x - nodes[mu]) / (nodes[nu] - nodes[mu])
    return out


def multi_indices(m: int) -> np.ndarray:
    """(K, 3) zero-based multi-indices, first axis slowest."""
    r = np.arange(m + 1)
    a, b, c = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)


def box_nodes_1d(lo: np.ndarray, hi: np.ndarray, m: int) -> np.ndarray:
    """Chebyshev nodes per axis of boxes: (nb, 3, m+1)."""
    x = chebyshev_nodes(m)
    lo = np.atleast_2d(lo)
    hi = np.atleast_2d(hi)
    return (0.5 * (lo + hi))[:, :, None] + (0.5 * (hi - lo))[:, :, None] * x


def box_nodes(lo: np.ndarray, hi: np.ndarray, m: int) -> np.ndarray:
    """Tensor nodes ``xi_{t,nu}`` of boxes: (nb, K, 3)."""
    n1 = box_nodes_1d(lo, hi, m)
    mi = multi_indices(m)
    return np.stack([n1[:, d, mi[:, d]] for d in range(3)], axis=2)


def interpolation_rows(points: np.ndarray, lo: np.ndarray, hi: np.ndarray,
                       m: int) -> np.ndarray:
    """``L_{t,nu}(x_j)`` for points ``x_j`` in boxes ``[lo, hi]``: (n, K).

    ``lo``/``hi`` give each point's own box, shape (n, 3).
    """
    points = np.atleast_2d(points)
    n1 = box_nodes_1d(lo, hi, m)  # (n, 3, m+1)
    mi = multi_indices(m)
    per_axis = []
    for d in range(3):
        vals = np.empty((points.shape[0], m + 1))
        for nu in range(m + 1):
            v = np.ones(points.shape[0])
            for mu in range(m + 1):
                if mu != nu:
                    v *= (points[:, d] - n1[:, d, mu]) / \
                        (n1[:, d, nu] - n1[:, d, mu])
            vals[:, nu] = v
        per_axis.append(vals)
    return per_axis[0][:, mi[:, 0]] * per_axis[1][:, mi[:, 1]] * \
        per_axis[2][:, mi[:, 2]]


def transfer_reference(m: int) -> np.ndarray:
    """The 8 non-directional transfer matrices ``E_{t'}`` (Sect. 2.7).

    Reference parent ``[-1,1]^3``; child octant ``q = 4*bx + 2*by + bz`` is
    the upper half along each axis with bit 1.  Returns (8, K, K) with
    ``E[q][j, k] = L_{t,nu_k}(xi_{t',nu_j})``.
    """
    lo = -np.ones((1, 3))
    hi = np.ones((1, 3))
    out = []
    for q in range(8):
        bits = np.array([(q >> 2) & 1, (q >> 1) & 1, q & 1])
        clo = np.where(bits == 1, 0.0, -1.0)[None, :]
        chi = np.where(bits == 1, 1.0, 0.0)[None, :]
        child_nodes = box_nodes(clo, chi, m)[0]  # (K, 3)
        K = child_nodes.shape[0]
        rows = interpolation_rows(child_nodes, np.repeat(lo, K, 0),
                                  np.repeat(hi, K, 0), m)
        out.append(rows)
    return np.stack(out)


def directional_part(child_lo: np.ndarray, child_hi: np.ndarray, m: int,
                     kappa: float, c: np.ndarray, cp: np.ndarray) -> np.ndarray:
    """Diagonals of ``E^d_{t',c}``: (nb, K) with ``exp(i k <xi_{t',nu}, c-c'>)``."""
    xi = box_nodes(child_lo, child_hi, m)  # (nb, K, 3)
    dc = np.asarray(c, dtype=np.float64) - np.asarray(cp, dtype=np.float64)
    return np.exp(1j * kappa * (xi @ dc))


def coupling_matrix(m: int, h: np.ndarray, o: np.ndarray, kappa: float,
                    c: np.ndarray) -> np.ndarray:
    """``A_{c,t x s}`` for same-level boxes of side ``h`` with ``m_t - m_s =
    h * o``: (K, K), rows over target nodes, columns over source nodes."""
    x = chebyshev_nodes(m)
    mi = multi_indices(m)
    h = np.asarray(h, dtype=np.float64)
    # node offsets from the box centre, per axis: (K, 3)
    rel = np.stack([0.5 * h[d] * x[mi[:, d]] for d in range(3)], axis=1)
    diff = (h * np.asarray(o, dtype=np.float64))[None, None, :] + \
        rel[:, None, :] - rel[None, :, :]  # xi_t,j - xi_s,k
    r = np.sqrt(np.sum(diff * diff, axis=2))
    phase = kappa * (r - diff @ np.asarray(c, dtype=np.float64))
    return np.exp(1j * phase) / (4.0 * np.pi * r)
