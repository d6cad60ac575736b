"""Adaptive trees in the oracle (Alg. 1 with n_max, Alg. 2 on unbalanced
trees, Alg. 4 with leaves on several levels), pinned against things other
than the code under test: the stop rule of Alg. 1, the printed recursion of
Alg. 2 and the partition property of its leaves (Sect. 2.3), the uniform
trees (n_max = 0), the dense product (a single leaf) and convergence in the
interpolation degree against the dense product."""
import numpy as np
import pytest

import oracle
import workloads as W


def clustered(seed, n, kappa, levels, m):
    rng = np.random.default_rng(seed)
    pt = W.clustered_points(rng, n)
    ps = W.clustered_points(rng, n)
    v = W.complex_normal(rng, n)
    return pt, ps, v, kappa, levels, m


@pytest.mark.parametrize("n_max", [0, 3, 10, 40])
def test_tree_follows_the_stop_rule(n_max):
    pt = clustered(1, 400, 10.0, 5, 2)[0]
    T = oracle.build_box_tree(pt, W.UNIT_BOX, 5, n_max)
    covered = np.zeros(T.n, dtype=np.int64)
    for l in range(T.levels + 1):
        leaf = T.is_leaf(l)
        # refined boxes hold more than n_max points; leaves at most n_max
        # unless they sit on the last level
        assert np.all(T.count[l][~leaf] > n_max)
        if l < T.levels:
            assert np.all(T.count[l][leaf] <= n_max)
        for b in np.flatnonzero(leaf):
            covered[T.start[l][b]:T.start[l][b] + T.count[l][b]] += 1
        if l:  # children tile their parent's points
            assert np.array_equal(np.bincount(T.parent[l], weights=T.count[l],
                                              minlength=T.keys[l - 1].shape[0]),
                                  np.where(T.is_leaf(l - 1), 0, T.count[l - 1]))
    assert np.all(covered == 1)  # leaves partition the points


def test_n_max_zero_is_the_uniform_tree():
    pt, ps, v, kappa, levels, m = clustered(2, 300, 15.0, 4, 2)
    a = oracle.build(pt, ps, kappa, W.UNIT_BOX, levels, m, n_max=0)
    b = oracle.build(pt, ps, kappa, W.UNIT_BOX, levels, m)
    sa, sb = oracle.structure(a), oracle.structure(b)
    assert sa.keys() == sb.keys()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(oracle.matvec(a, v), oracle.matvec(b, v))


def test_single_leaf_is_the_dense_product():
    """n_max >= N: the root is a leaf, the block tree is the one inadmissible
    root block, and Alg. 4 is the dense product."""
    pt, ps, v, kappa, levels, m = clustered(3, 250, 25.0, 4, 3)
    plan = oracle.build(pt, ps, kappa, W.UNIT_BOX, levels, m, n_max=250)
    assert plan.TT.keys[1].size == 0 and plan.BT.near_t[0].size == 1
    y = oracle.matvec(plan, v)
    yd = oracle.dense_matvec(pt, ps, v, kappa)
    assert np.linalg.norm(y - yd) <= 1e-13 * np.linalg.norm(yd)


def _literal_blocks(TT, TS, kappa):
    """Alg. 2 as printed: depth-first from the pair of roots; a pair with a
    leaf on either side is a leaf block."""
    adm, near = [], []

    def refine(level, t, s):
        o = TT.coords[level][t] - TS.coords[level][s]
        ok = bool(oracle.admissible(kappa, TT.side(level), o))
        if TT.child_count[level][t] == 0 or TS.child_count[level][s] == 0:
            (adm if ok else near).append((level, t, s))
            return
        if ok:
            adm.append((level, t, s))
            return
        for tc in range(TT.child_start[level][t],
                        TT.child_start[level][t] + TT.child_count[level][t]):
            for sc in range(TS.child_start[level][s],
                            TS.child_start[level][s] + TS.child_count[level][s]):
                refine(level + 1, tc, sc)

    refine(0, 0, 0)
    return sorted(adm), sorted(near)


@pytest.mark.parametrize("n_max", [2, 6, 20])
def test_block_tree_matches_alg2_and_partitions(n_max):
    pt, ps, v, kappa, levels, m = clustered(4, 150, 20.0, 4, 2)
    TT = oracle.build_box_tree(pt, W.UNIT_BOX, levels, n_max)
    TS = oracle.build_box_tree(ps, W.UNIT_BOX, levels, n_max)
    BT = oracle.block_tree(TT, TS, kappa)
    adm = sorted((l, int(t), int(s)) for l in range(levels + 1)
                 for t, s in zip(BT.adm_t[l], BT.adm_s[l]))
    near = sorted((l, int(t), int(s)) for l in range(levels + 1)
                  for t, s in zip(BT.near_t[l], BT.near_s[l]))
    ladm, lnear = _literal_blocks(TT, TS, kappa)
    assert adm == ladm and near == lnear
    assert len({l for l, _, _ in near}) >= 2  # near field on several levels
    cover = np.zeros((TT.n, TS.n), dtype=np.int64)
    for (l, t, s) in adm + near:
        cover[TT.start[l][t]:TT.start[l][t] + TT.count[l][t],
              TS.start[l][s]:TS.start[l][s] + TS.count[l][s]] += 1
    assert np.all(cover == 1)


def test_adaptive_product_converges_to_the_dense_one():
    """Clustered points, n_max = 8: the error against the dense product falls
    with the degree m as for uniform trees (interpolation error), and the
    leaves and near-field blocks really sit on several levels."""
    pt, ps, v, kappa, levels, m = clustered(5, 400, 15.0, 5, 2)
    yd = oracle.dense_matvec(pt, ps, v, kappa)
    errs = []
    for m in (2, 4):
        plan = oracle.build(pt, ps, kappa, W.UNIT_BOX, levels, m, n_max=8)
        y = oracle.matvec(plan, v)
        errs.append(np.linalg.norm(y - yd) / np.linalg.norm(yd))
    assert len([l for l in range(levels + 1) if plan.TT.is_leaf(l).any()]) >= 3
    assert len([l for l in range(levels + 1) if plan.BT.near_t[l].size]) >= 2
    assert errs[1] < errs[0] / 10 and errs[1] < 1e-3, errs


def test_sampled_rows_match_the_full_product():
    pt, ps, v, kappa, levels, m = clustered(6, 300, 12.0, 4, 3)
    full = oracle.matvec(oracle.build(pt, ps, kappa, W.UNIT_BOX, levels, m, n_max=5), v)
    rows = np.random.default_rng(0).choice(300, 25, replace=False)
    y = oracle.sample_rows(pt, ps, v, kappa, W.UNIT_BOX, levels, m, rows, n_max=5)
    assert np.linalg.norm(y - full[rows]) <= 1e-13 * np.linalg.norm(full[rows])


def test_invalid_n_max():
    pt, ps, v, kappa, levels, m = clustered(7, 20, 5.0, 2, 2)
    for bad in (-1, 2.5):
        with pytest.raises(ValueError):
            oracle.build(pt, ps, kappa, W.UNIT_BOX, levels, m, n_max=bad)
