"""Pins of the oracle's interpolation operators and of Alg. 4 (CPU only)."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.interpolation import (box_nodes, box_nodes_1d, directional_part,
                                  lagrange_1d)


# ------------------------------------------------- Chebyshev / Lagrange --
@pytest.mark.parametrize("m", [1, 2, 4, 6, 8])
def test_chebyshev_nodes_are_roots(m):
    x = oracle.chebyshev_nodes(m)
    assert np.all(np.diff(x) < 0)  # nu = 1..m+1 descending
    T = np.cos((m + 1) * np.arccos(x))  # T_{m+1}(x_nu) = 0
    assert np.max(np.abs(T)) < 1e-14
    # against numpy's Chebyshev root finder
    roots = np.polynomial.chebyshev.chebroots([0] * (m + 1) + [1])
    assert np.allclose(np.sort(roots), np.sort(x), atol=1e-13)


@pytest.mark.parametrize("m", [2, 4, 6])
def test_lagrange_partition_of_unity_and_cardinal(m):
    x = oracle.chebyshev_nodes(m)
    L = lagrange_1d(x, np.linspace(-1, 1, 37))
    assert np.allclose(L.sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(lagrange_1d(x, x), np.eye(m + 1), atol=1e-14)


@pytest.mark.parametrize("m", [3, 5])
def test_tensor_interpolation_reproduces_polynomials(m):
    """Degree <= m per axis is reproduced exactly (Sect. 2.2)."""
    rng = np.random.default_rng(m)
    coef = rng.standard_normal((m + 1, m + 1, m + 1))
    poly = lambda P: np.polynomial.polynomial.polyval3d(P[:, 0], P[:, 1], P[:, 2], coef)
    lo, hi = np.array([0.25, -0.5, 1.0]), np.array([0.75, 0.0, 1.5])
    nodes = box_nodes(lo[None], hi[None], m)[0]  # (K, 3)
    pts = lo + (hi - lo) * rng.random((50, 3))
    L = oracle.interpolation_rows(pts, np.repeat(lo[None], 50, 0),
                                  np.repeat(hi[None], 50, 0), m)
    assert np.allclose(L @ poly(nodes), poly(pts), rtol=1e-11, atol=1e-11)
    # a polynomial of degree m+1 is not reproduced
    coef2 = np.zeros((m + 2, 1, 1))
    coef2[m + 1, 0, 0] = 1.0
    poly2 = lambda P: np.polynomial.polynomial.polyval3d(P[:, 0], P[:, 1], P[:, 2], coef2)
    assert not np.allclose(L @ poly2(nodes), poly2(pts), atol=1e-6)


def test_multi_index_order_first_axis_slowest():
    mi = oracle.multi_indices(2)
    assert mi[:4].tolist() == [[0, 0, 0], [0, 0, 1], [0, 0, 2], [0, 1, 0]]
    assert mi[9].tolist() == [1, 0, 0]


@pytest.mark.parametrize("m", [2, 4])
def test_transfer_reference_maps_parent_to_child_values(m):
    """E_{t'} interpolates parent nodal values of a degree-m polynomial to
    the child nodes exactly; there are exactly 8 such matrices (Sect. 2.7)."""
    E = oracle.transfer_reference(m)
    assert E.shape == (8, (m + 1) ** 3, (m + 1) ** 3)
    assert len({E[q].tobytes() for q in range(8)}) == 8
    rng = np.random.default_rng(1)
    coef = rng.standard_normal((m + 1,) * 3)
    poly = lambda P: np.polynomial.polynomial.polyval3d(P[:, 0], P[:, 1], P[:, 2], coef)
    pn = box_nodes(-np.ones((1, 3)), np.ones((1, 3)), m)[0]
    for q in range(8):
        bits = np.array([(q >> 2) & 1, (q >> 1) & 1, q & 1])
        cn = box_nodes(np.where(bits, 0.0, -1.0)[None], np.where(bits, 1.0, 0.0)[None], m)[0]
        assert np.allclose(E[q] @ poly(pn), poly(cn), atol=1e-11)


# --------------------------------------------------------------- kernel --
def test_helmholtz_kernel_values():
    r = np.array([0.5, 1.0, 0.0])
    f = oracle.helmholtz(r, 3.0)
    assert f[2] == 0
    assert np.isclose(f[0], (np.cos(1.5) + 1j * np.sin(1.5)) / (2 * np.pi), rtol=1e-15)
    assert np.isclose(f[1], (np.cos(3.0) + 1j * np.sin(3.0)) / (4 * np.pi), rtol=1e-15)


def test_coupling_depends_only_on_offset_and_transposes():
    m, kappa = 3, 17.0
    h = np.full(3, 0.125)
    o = np.array([4, -1, 2])
    c = np.array([1.0, -0.25, 0.5]) / np.linalg.norm([1.0, -0.25, 0.5])
    A = oracle.coupling_matrix(m, h, o, kappa, c)
    # direct definition f_c(xi_t, xi_s) on two different pairs of boxes
    for base in (np.array([0.0, 0.5, 0.25]), np.array([0.375, 0.125, 0.0])):
        ts_lo = base + o * h
        xt = box_nodes(ts_lo[None], (ts_lo + h)[None], m)[0]
        xs = box_nodes(base[None], (base + h)[None], m)[0]
        d = xt[:, None, :] - xs[None, :, :]
        r = np.linalg.norm(d, axis=2)
        direct = np.exp(1j * kappa * (r - d @ c)) / (4 * np.pi * r)
        assert np.allclose(A, direct, rtol=1e-13, atol=0)
    # swapping the roles of t and s: A_{-c, -o} = A_{c, o}^T
    B = oracle.coupling_matrix(m, h, -o, kappa, -c)
    assert np.allclose(B, A.T, rtol=1e-13)


def test_directional_part_is_identity_for_equal_directions():
    lo = np.array([[0.0, 0.25, 0.5]])
    Ed = directional_part(lo, lo + 0.25, 3, 50.0, np.array([0.0, 0, 1]), np.array([0.0, 0, 1]))
    assert np.allclose(Ed, 1.0)


# ---------------------------------------------------------------- Alg. 4 --
def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("levels", [0, 1])
def test_no_admissible_blocks_means_dense(levels):
    P = W.random_problem(4, 300, 280, 25.0, levels, 3)
    y = oracle.matvec(oracle.build(P.points_T, P.points_S, P.kappa, P.box, levels, 3), P.v)
    yd = oracle.dense_matvec(P.points_T, P.points_S, P.v, P.kappa)
    assert _rel(y, yd) < 1e-14


def test_converges_to_dense_with_m():
    """Exponential convergence in m (Sect. 2.2); 2000 uniform points."""
    P = W.random_problem(8, 900, 800, 20.0, 3, 2)
    yd = oracle.dense_matvec(P.points_T, P.points_S, P.v, P.kappa)
    errs = []
    for m in (2, 3, 4):
        plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, 3, m)
        assert plan.BT.n_admissible() > 0
        errs.append(_rel(oracle.matvec(plan, P.v), yd))
    assert all(b < 0.35 * a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 2e-3


def test_laplace_limit():
    """kappa = 0: no directions, the Laplace kernel 1/(4 pi r); nested
    interpolation is exact for polynomials, so the error is the plain
    interpolation error and falls with m."""
    P = W.random_problem(9, 1000, 900, 0.0, 3, 2)
    yd = oracle.dense_matvec(P.points_T, P.points_S, P.v, 0.0)
    # kappa = 0 gives the real kernel 1/(4 pi r): real charges, real result
    assert np.all(oracle.dense_matvec(P.points_T[:50], P.points_S, P.v.real, 0.0).imag == 0)
    errs = []
    for m in (2, 4, 6):
        plan = oracle.build(P.points_T, P.points_S, 0.0, P.box, 3, m)
        assert plan.l_hf == -1
        errs.append(_rel(oracle.matvec(plan, P.v), yd))
    assert errs[0] > 10 * errs[1] > 100 * errs[2]


def test_nested_moments_equal_direct_moments_low_frequency():
    """On low-frequency levels L_{s,nu} is a degree-m polynomial, so M2M of
    the leaf moments equals the S2M of the parent box exactly (Sect. 2.5)."""
    P = W.random_problem(12, 400, 500, 0.0, 3, 3)
    plan = oracle.build(P.points_T, P.points_S, 0.0, P.box, 3, 3)
    oracle.matvec(plan, P.v, keep=True)
    mom = plan.debug["mom"]
    TS = plan.TS
    vt = P.v[TS.perm]
    for level in (1, 2):
        need = plan.DS[level][:, 0] | plan.DhS[level][:, 0]
        for s in np.flatnonzero(need)[:10]:
            sl = slice(TS.start[level][s], TS.start[level][s] + TS.count[level][s])
            n = TS.count[level][s]
            L = oracle.interpolation_rows(TS.points[sl], np.repeat(TS.lo[level][s][None], n, 0),
                                          np.repeat(TS.hi[level][s][None], n, 0), 3)
            direct = L.T @ vt[sl]
            assert np.allclose(mom[level][s, 0], direct, rtol=1e-11, atol=1e-11)


def test_symmetry_of_the_approximant():
    """A(S,T) = A(T,S)^T (f is symmetric); with dir(-v) = -dir(v) the
    approximation keeps it: u^T A~(T,S) v = v^T A~(S,T) u."""
    P = W.random_problem(14, 700, 650, 30.0, 3, 3)
    rng = np.random.default_rng(3)
    u = W.complex_normal(rng, 700)
    pts = oracle.build(P.points_T, P.points_S, P.kappa, P.box, 3, 3)
    pst = oracle.build(P.points_S, P.points_T, P.kappa, P.box, 3, 3)
    assert pts.l_hf >= 1 and pts.BT.n_admissible() > 0
    a = u @ oracle.matvec(pts, P.v)
    b = P.v @ oracle.matvec(pst, u)
    assert abs(a - b) <= 1e-13 * abs(a)


def test_sample_rows_equal_full_rows():
    P = W.config("uniform2k")
    plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m)
    y = oracle.matvec(plan, P.v)
    rows = np.array([3, 400, 1234, 1999, 3])
    ys = oracle.sample_rows(P.points_T, P.points_S, P.v, P.kappa, P.box, P.levels, P.m, rows)
    assert np.allclose(ys, y[rows], rtol=1e-13, atol=1e-13 * np.abs(y).max())


def test_uniform2k_against_dense():
    """2000 points, kappa 20, 3 levels, m=4: the approximation error of the
    method (no bound printed in the paper; measured 6.0e-4)."""
    P = W.config("uniform2k")
    plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m)
    y = oracle.matvec(plan, P.v)
    yd = oracle.dense_matvec(P.points_T, P.points_S, P.v, P.kappa)
    assert 1e-5 < _rel(y, yd) < 2e-3


def test_paper_k6_error_matches_printed_value():
    """Sect. 4: relative error about 2e-4 for k=6, m=4 (the paper's code also
    compresses couplings by ACA, so ours may only be smaller, not much).
    Measured on 256 sampled rows against the dense rows: 1.75e-4."""
    P = W.config("paper_k6")
    rows = np.random.default_rng(0).choice(P.points_T.shape[0], 256, replace=False)
    plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m, rows=rows)
    y = oracle.matvec(plan, P.v)
    yd = oracle.dense_rows(P.points_T, P.points_S, P.v, P.kappa, rows)
    err = _rel(y, yd)
    assert 2e-4 / 3 < err < 2e-4 * 1.5


def test_dense_rows_brute_force_with_coinciding_point():
    """The dense product (Sect. 1) against a scalar double loop with
    math.cos / math.sin, including a target equal to a source (zero term)
    and a chunk size that leaves a ragged last chunk."""
    import math
    rng = np.random.default_rng(9)
    X = rng.uniform(-1, 1, (7, 3))
    Y = rng.uniform(-1, 1, (9, 3))
    Y[4] = X[2]
    v = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    kappa = 6.5
    want = []
    for x in X:
        s = 0j
        for yk, vk in zip(Y, v):
            r = math.sqrt(sum((a - b) ** 2 for a, b in zip(x, yk)))
            if r > 0:
                s += complex(math.cos(kappa * r), math.sin(kappa * r)) / (4 * math.pi * r) * vk
        want.append(s)
    want = np.array(want)
    for chunk in (2, 256):
        got = oracle.dense_rows(X, Y, v, kappa, np.arange(7), chunk=chunk)
        assert np.allclose(got, want, rtol=1e-13, atol=0)


@pytest.mark.parametrize("name", ["uniform100k", "uniform1m"])
def test_stored_rows_approximate_the_dense_product(name):
    """The stored oracle rows of the full-size workloads (written by
    tests/golden/make_golden.py) against the dense sum (Sect. 1) at the same
    rows: within the method's approximation error for these m and kappa,
    and not equal to it (they are the fast method's values)."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", f"{name}_rows.npz"))
    P = W.config(name)
    yd = oracle.dense_rows(P.points_T, P.points_S, P.v, P.kappa, g["rows"])
    err = np.linalg.norm(g["y"] - yd) / np.linalg.norm(yd)
    assert 1e-6 < err < 1e-3, err


def test_stored_batch_rows_approximate_the_dense_product():
    """As above for the four stored problems of the batched workload (two
    uniform, two clustered)."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "batch_rows.npz"))
    probs = W.batch_problems()
    for i in (2, 4, 35, 46):
        P = probs[i]
        yd = oracle.dense_rows(P.points_T, P.points_S, P.v, P.kappa, g[f"rows{i}"])
        err = np.linalg.norm(g[f"y{i}"] - yd) / np.linalg.norm(yd)
        assert 1e-6 < err < 2e-3, (i, err)
