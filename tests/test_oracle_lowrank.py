"""Pins of the oracle's adaptive cross approximation (Sect. 2.7): exact
recovery of matrices of known rank, the error on the Helmholtz coupling
matrices against the tolerance and against the best error of that rank
(SVD), and the matvec with compressed couplings against the dense-coupling
matvec."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.interpolation import coupling_matrix


def _rel(A, B):
    return np.linalg.norm(A - B) / np.linalg.norm(B)


@pytest.mark.parametrize("shape,r", [((40, 30), 1), ((64, 64), 6), ((50, 80), 12)])
def test_exact_low_rank_recovery(shape, r):
    rng = np.random.default_rng(7 + r)
    X = rng.standard_normal((shape[0], r)) + 1j * rng.standard_normal((shape[0], r))
    Y = rng.standard_normal((shape[1], r)) + 1j * rng.standard_normal((shape[1], r))
    A = X @ Y.conj().T
    U, Wm = oracle.aca_dense(A, 1e-13)
    assert U.shape[1] <= r + 1
    assert _rel(U @ Wm.conj().T, A) <= 1e-12


def test_zero_rows_and_zero_matrix():
    rng = np.random.default_rng(3)
    A = np.zeros((20, 15), dtype=np.complex128)
    A[7:] = np.outer(rng.standard_normal(13), rng.standard_normal(15))  # rows 0..6 zero
    U, Wm = oracle.aca_dense(A, 1e-12)
    assert U.shape[1] <= 2 and _rel(U @ Wm.conj().T, A) <= 1e-13  # last cross ~ roundoff
    U0, W0 = oracle.aca_dense(np.zeros((5, 4), dtype=np.complex128), 1e-12)
    assert U0.shape == (5, 0) and W0.shape == (4, 0)


@pytest.mark.parametrize("eps", [1e-4, 1e-8])
@pytest.mark.parametrize("o,c", [((3, 0, 0), (1.0, 0.0, 0.0)), ((2, 2, 1), (0.0, 0.0, 0.0)),
                                 ((4, -3, 2), (0.6, -0.48, 0.64))])
def test_coupling_matrices_within_tolerance(o, c, eps):
    """Smooth kernels: the compressed coupling matrix is within a small
    multiple of eps, its rank below K, and its error within a small factor of
    the SVD's best error at the same rank."""
    m, h, kappa = 5, np.full(3, 0.125), 40.0
    c = np.asarray(c) / max(np.linalg.norm(c), 1.0)
    A = coupling_matrix(m, h, np.asarray(o, float), kappa, c)
    U, Wm = oracle.aca_dense(A, eps)
    k = U.shape[1]
    err = _rel(U @ Wm.conj().T, A)
    assert err <= 20 * eps
    assert k < A.shape[0]
    s = np.linalg.svd(A, compute_uv=False)
    best = np.sqrt(np.sum(s[k:] ** 2)) / np.sqrt(np.sum(s ** 2))
    assert err <= max(20 * best, 1e-15)
    assert k >= int(np.sum(s > 1e-3 * eps * s[0])) // 4  # not absurdly small either


def test_matvec_with_compressed_couplings():
    P = W.random_problem(51, 700, 650, 40.0, 3, 4)
    plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m)
    epss = (1e-4, 1e-6, 1e-10)
    ys = oracle.matvec(plan, P.v, m2l=("fp64",) + tuple(f"aca:{e:g}" for e in epss))
    for eps, ya in zip(epss, ys[1:]):
        # the operator error follows the tolerance (about 0.4 eps here), and
        # is not zero: the compressed matrices are the ones applied
        assert 0.05 * eps <= _rel(ya, ys[0]) <= 2 * eps, eps
