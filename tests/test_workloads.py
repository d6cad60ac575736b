"""The seeded input generators: reproducible draws, every point inside its
half-open box (lo, hi] (the library rejects others), and the stated recipe
of each workload (sizes, wave numbers, depths, the grid of Sect. 4, the
batched mix)."""
import numpy as np
import pytest

import workloads as W


def _inside(P):
    lo, hi = np.asarray(P.box[:3]), np.asarray(P.box[3:])
    for pts in (P.points_T, P.points_S):
        assert np.all(pts > lo) and np.all(pts <= hi)


@pytest.mark.parametrize("name", ["uniform2k", "uniform100k", "uniform1m", "paper_k5"])
def test_named_workloads(name):
    P = W.config(name)
    Q = W.config(name)
    assert np.array_equal(P.points_T, Q.points_T) and np.array_equal(P.v, Q.v)
    _inside(P)
    if name in W.UNIFORM:
        seed, n, kappa, levels, m = W.UNIFORM[name]
        assert P.points_T.shape == (n, 3) and P.points_S.shape == (n, 3)
        assert (P.kappa, P.levels, P.m) == (kappa, levels, m)
        assert not np.array_equal(P.points_T, P.points_S)
        assert abs(P.v.real.std() - 1) < 0.05 and abs(P.v.imag.std() - 1) < 0.05
    else:  # Sect. 4: 8^k grid points, kappa = 0.1 * 2^k, depth k - 3
        k = 5
        assert P.points_T.shape == (8 ** k, 3) and P.same_points
        assert P.kappa == 0.1 * 2 ** k and P.levels == k - 3
        x = np.unique(P.points_T[:, 0])
        assert np.allclose(np.diff(x), 2.0 ** (1 - k)) and np.isclose(x[0], 2.0 ** -k - 1)


def test_random_and_clustered_problems():
    for P in (W.random_problem(3, 500, 400, 10.0, 3, 3, (-2.0, 1.0, 0.5, 2.0, 5.0, 4.5)),
              W.clustered_problem(4, 5000, 4000, 10.0, 3, 3)):
        _inside(P)
        assert P.points_T.shape[0] != P.points_S.shape[0]
    C = W.clustered_problem(4, 5000, 4000, 10.0, 3, 3)
    # blobs of sigma 0.05: most leaves of a 3-level tree are empty
    keys = np.unique(np.floor(C.points_T * 8).astype(int), axis=0)
    assert keys.shape[0] < 0.5 * 8 ** 3


def test_batched_workload_recipe():
    probs = W.batch_problems()
    assert len(probs) == 64
    n = np.array([p.points_T.shape[0] for p in probs])
    assert n.min() >= 1e4 and n.max() <= 2e5
    assert all(10 <= p.kappa <= 80 for p in probs)
    assert [p.meta["kind"] for p in probs] == ["uniform"] * 32 + ["clustered"] * 32
    for p in probs:
        _inside(p)
        assert p.levels == W.batch_levels(p.points_T.shape[0])
        assert np.array_equal(p.v.astype(np.complex64).astype(np.complex128), p.v)
    again = W.batch_problems()
    assert all(np.array_equal(a.points_S, b.points_S) for a, b in zip(probs, again))
