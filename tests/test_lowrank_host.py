"""The library's adaptive cross approximation (``fdm_aca``, Sect. 2.7; host
code, so these run without a GPU) against the oracle's: the same crosses
(rank, pivots, vectors to rounding) on random low-rank matrices and on the
Helmholtz coupling matrices, plus the properties that pin both (exact
recovery, the tolerance, the rank cap, zero rows) and argument checks."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2004_14229_amd as F
from oracle.interpolation import coupling_matrix


def _rel(A, B):
    return np.linalg.norm(A - B) / max(np.linalg.norm(B), 1e-300)


def _low_rank(seed, n, m, r):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    Y = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    return X @ Y.conj().T


def _size(U, W, l):
    return np.linalg.norm(U[:, l]) * np.linalg.norm(W[:, l])


def _same_crosses(A, eps, max_rank=None):
    """Both ACAs take the same crosses: each cross u_l v_l^T agrees to 1e-10
    of |A|_F (so the same pivots), and the ranks agree except for a last
    cross at round-off level (whose pivot round-off decides)."""
    U, Wm = F.aca(A, eps, max_rank)
    Uo, Wo = oracle.aca_dense(A, eps, max_rank)
    nA = np.linalg.norm(A)
    k, ko = U.shape[1], Uo.shape[1]
    assert abs(k - ko) <= 1
    assert all(_size(U, Wm, l) <= 1e-12 * nA for l in range(ko, k))
    assert all(_size(Uo, Wo, l) <= 1e-12 * nA for l in range(k, ko))
    for l in range(min(k, ko)):
        d = np.outer(U[:, l], Wm[:, l].conj()) - np.outer(Uo[:, l], Wo[:, l].conj())
        assert np.linalg.norm(d) <= 1e-10 * nA, l
        if _size(U, Wm, l) > 1e-12 * nA:  # v_l is scaled to 1 at its pivot column
            assert abs(np.abs(Wm[:, l]).max() - 1.0) <= 1e-15
    return U, Wm


@pytest.mark.parametrize("shape,r", [((40, 30), 1), ((64, 64), 6), ((50, 80), 12),
                                     ((7, 200), 5)])
def test_exact_low_rank_recovery(shape, r):
    A = _low_rank(11 + r, *shape, r)
    U, Wm = _same_crosses(A, 1e-13)
    assert U.shape[1] <= r + 1
    assert _rel(U @ Wm.conj().T, A) <= 1e-12


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-10])
@pytest.mark.parametrize("o,c", [((3, 0, 0), (1.0, 0.0, 0.0)), ((2, 2, 1), (0.0, 0.0, 0.0)),
                                 ((4, -3, 2), (0.6, -0.48, 0.64)), ((0, 5, -2), (0, 1, 0))])
def test_coupling_matrices_match_oracle(o, c, eps):
    m, h, kappa = 5, np.full(3, 0.125), 40.0
    c = np.asarray(c, float) / max(np.linalg.norm(c), 1.0)
    A = coupling_matrix(m, h, np.asarray(o, float), kappa, c)
    U, Wm = _same_crosses(A, eps)
    assert U.shape[1] < A.shape[0]
    assert _rel(U @ Wm.conj().T, A) <= 20 * eps


def test_rank_cap_and_full_rank():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((30, 24)) + 1j * rng.standard_normal((30, 24))
    U, Wm = _same_crosses(A, 0.0, 7)
    assert U.shape == (30, 7) and Wm.shape == (24, 7)
    U, Wm = _same_crosses(A, 0.0)  # eps 0: crosses until every column is spent
    assert U.shape[1] == 24 and _rel(U @ Wm.conj().T, A) <= 1e-12


def test_zero_rows_and_zero_matrix():
    rng = np.random.default_rng(3)
    A = np.zeros((20, 15), dtype=np.complex128)
    A[7:] = np.outer(rng.standard_normal(13), rng.standard_normal(15))  # rows 0..6 zero
    U, Wm = _same_crosses(A, 1e-12)
    assert U.shape[1] <= 2 and _rel(U @ Wm.conj().T, A) <= 1e-13
    U0, W0 = F.aca(np.zeros((5, 4), dtype=np.complex128), 1e-12)
    assert U0.shape == (5, 0) and W0.shape == (4, 0)


def test_single_row_and_column():
    a = np.arange(1, 9) * (1 + 0.5j)
    for A in (a[None, :], a[:, None]):
        U, Wm = _same_crosses(A, 1e-14)
        assert U.shape[1] == 1 and _rel(U @ Wm.conj().T, A) <= 1e-15


def _raw(A, eps, max_rank, U=None, W=None):
    L = F.lib()
    n, m = A.shape
    U = np.zeros((n, max(max_rank, 1)), np.complex128) if U is None else U
    W = np.zeros((m, max(max_rank, 1)), np.complex128) if W is None else W
    k = ctypes.c_int(-7)
    st = L.fdm_aca(A.ctypes.data, n, m, eps, max_rank, U.ctypes.data, W.ctypes.data,
                   ctypes.byref(k))
    return st, k.value, L.fdm_last_error().decode()


def test_invalid_arguments():
    L = F.lib()
    A = np.ones((4, 3), np.complex128)
    for eps, R in ((-1.0, 2), (float("nan"), 2), (float("inf"), 2), (1e-8, 0), (1e-8, 4)):
        st, k, msg = _raw(A, eps, R)
        assert st == -1 and k == -7 and msg, (eps, R)
    assert L.fdm_aca(None, 4, 3, 1e-8, 2, None, None, None) == -1
    U = np.zeros((4, 2), np.complex128)
    W = np.zeros((3, 2), np.complex128)
    k = ctypes.c_int()
    assert L.fdm_aca(A.ctypes.data, 0, 3, 1e-8, 1, U.ctypes.data, W.ctypes.data,
                     ctypes.byref(k)) == -1
    B = A.copy()
    B[2, 1] = np.nan
    st, k, msg = _raw(B, 1e-8, 2)
    assert st == -1 and "non-finite" in msg


def test_unused_columns_are_zeroed():
    A = _low_rank(9, 12, 10, 2)
    U = np.full((12, 6), 3 + 3j)
    W = np.full((10, 6), 3 + 3j)
    st, k, _ = _raw(A, 1e-13, 6, U, W)
    assert st == 0 and 2 <= k <= 3
    assert np.all(U[:, k:] == 0) and np.all(W[:, k:] == 0)
    assert _rel(U[:, :k] @ W[:, :k].conj().T, A) <= 1e-12
