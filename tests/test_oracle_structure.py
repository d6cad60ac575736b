"""Pins of the oracle's tree, block tree and directions (CPU only).

Each test checks the oracle against something other than itself: the paper's
Table 1 (Sect. 4), closed forms, or a literal brute-force re-derivation on
tiny inputs.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.directions import DirectionSets


# ----------------------------------------------------------------- Alg. 1 --
def test_tree_cells_match_dyadic_closed_form():
    """In the unit cube the level-l cell of x is ceil(x 2^l) - 1 per axis."""
    rng = np.random.default_rng(11)
    pts = W.unit_cube_points(rng, 3000)
    T = oracle.build_box_tree(pts, W.UNIT_BOX, 5)
    inv = np.empty(T.n, dtype=np.int64)
    inv[T.perm] = np.arange(T.n)
    for level in range(6):
        cell = np.ceil(pts * 2.0 ** level).astype(np.int64) - 1
        box = np.repeat(np.arange(T.keys[level].shape[0]), T.count[level])
        assert np.array_equal(T.coords[level][box[inv]], cell)


def test_tree_points_inside_boxes_and_order():
    P = W.random_problem(3, 700, 10, 5.0, 4, 3, box=(-2.0, 1.0, 0.5, 2.0, 5.0, 4.5))
    T = oracle.build_box_tree(P.points_T, P.box, 4)
    for level in range(5):
        box = np.repeat(np.arange(T.keys[level].shape[0]), T.count[level])
        assert np.all(T.points > T.lo[level][box])
        assert np.all(T.points <= T.hi[level][box])
        assert np.all(np.diff(T.keys[level]) > 0)  # Morton order, unique
        assert T.count[level].sum() == 700
    # ties inside a leaf keep the input order
    p = T.levels
    for s, c in zip(T.start[p], T.count[p]):
        assert np.all(np.diff(T.perm[s:s + c]) > 0)
    assert np.array_equal(np.sort(T.perm), np.arange(700))


def test_tree_boundary_point_goes_to_lower_child():
    pts = np.array([[0.5, 0.25, 1.0], [0.5000000000000001, 0.75, 0.125]])
    T = oracle.build_box_tree(pts, W.UNIT_BOX, 2)
    inv = np.empty(2, dtype=np.int64)
    inv[T.perm] = np.arange(2)
    box = np.repeat(np.arange(T.keys[2].shape[0]), T.count[2])
    assert T.coords[2][box[inv[0]]].tolist() == [1, 0, 3]
    assert T.coords[2][box[inv[1]]].tolist() == [2, 2, 0]
    with pytest.raises(ValueError):
        oracle.build_box_tree(np.array([[0.0, 0.5, 0.5]]), W.UNIT_BOX, 2)


@pytest.mark.parametrize("k", [5, 6])
def test_paper_grid_is_uniform_octree(k):
    """Sect. 4: depth k-3, every leaf holds exactly 512 points."""
    pts = W.paper_grid_points(k)
    T = oracle.build_box_tree(pts, (-1, -1, -1, 1, 1, 1), k - 3)
    assert T.keys[k - 3].shape[0] == 8 ** (k - 3)
    assert np.all(T.count[k - 3] == 512)


# ---------------------------------------------- Def. (A1)-(A3), Alg. 2 --
def test_admissibility_ties_are_admissible():
    """kappa=20, level 2 of the unit cube: (kappa*D^2/eta2)^2 = 9 h^2-units
    is met exactly by g = (2,2,1); ties count as admissible."""
    h = np.full(3, 0.25)
    assert oracle.admissible(20.0, h, np.array([3, 3, 2]))
    assert oracle.admissible(20.0, h, np.array([-2, 3, 3]))
    assert not oracle.admissible(20.0, h, np.array([3, 3, 1]))
    assert not oracle.admissible(20.0, h, np.array([0, 0, 0]))


def test_admissibility_against_exact_geometry():
    """(A1)/(A3) evaluated with exact rational distances agree."""
    rng = np.random.default_rng(5)
    for _ in range(400):
        level = int(rng.integers(0, 6))
        h = Fraction(1, 2 ** level)
        kappa = int(rng.integers(0, 60))
        o = rng.integers(-9, 10, size=3)
        g = [max(abs(int(x)) - 1, 0) for x in o]
        d2 = 3 * h * h
        s2 = sum((gi * h) ** 2 for gi in g)
        exact = (d2 <= 25 * s2) and (kappa * kappa * d2 * d2 <= 25 * s2)
        got = bool(oracle.admissible(float(kappa), np.full(3, float(h)), o))
        assert got == exact


def _literal_block_tree(TT, TS, kappa):
    """Alg. 2 as printed: depth-first recursion from the pair of roots."""
    adm, near = [], []

    def refine(level, t, s):
        o = TT.coords[level][t] - TS.coords[level][s]
        ok = bool(oracle.admissible(kappa, TT.side(level), o))
        if TT.child_count[level][t] == 0 or TS.child_count[level][s] == 0:
            (adm if ok else near).append((level, t, s))  # t or s is a leaf
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


def test_block_tree_matches_literal_recursion_and_partitions():
    P = W.random_problem(7, 90, 70, 20.0, 3, 2)
    TT = oracle.build_box_tree(P.points_T, P.box, 3)
    TS = oracle.build_box_tree(P.points_S, P.box, 3)
    BT = oracle.block_tree(TT, TS, P.kappa)
    adm = sorted((l, int(t), int(s)) for l in range(4)
                 for t, s in zip(BT.adm_t[l], BT.adm_s[l]))
    near = sorted((3, int(t), int(s)) for t, s in zip(BT.near_t[3], BT.near_s[3]))
    ladm, lnear = _literal_block_tree(TT, TS, P.kappa)
    assert adm == ladm and near == lnear
    # the leaves partition the index set {1..N_T} x {1..N_S} (Sect. 2.3)
    cover = np.zeros((TT.n, TS.n), dtype=np.int64)
    for (l, t, s) in ladm + lnear:
        cover[TT.start[l][t]:TT.start[l][t] + TT.count[l][t],
              TS.start[l][s]:TS.start[l][s] + TS.count[l][s]] += 1
    assert np.all(cover == 1)


def _table1_counts(k):
    """Block-tree counts for the full grid of Sect. 4 by offset recursion."""
    p, kappa = k - 3, 0.1 * 2.0 ** k
    cnt = np.ones((1, 1, 1), dtype=np.int64)  # level 0: the root pair
    nc = nsc = 0
    w = {-1: 1, 0: 2, 1: 1}
    for level in range(p + 1):
        r = (cnt.shape[0] - 1) // 2
        o = np.stack(np.meshgrid(*[np.arange(-r, r + 1)] * 3, indexing="ij"), -1)
        adm = oracle.admissible(kappa, np.full(3, 2.0 * 2.0 ** (-level)), o)
        nc += int(cnt[adm].sum())
        nsc += int(np.count_nonzero(cnt[adm]))
        if level == p:
            near = int(cnt[~adm].sum())
            break
        ref = np.where(adm, 0, cnt)
        R = 2 ** (level + 1) - 1
        child = np.zeros((2 * R + 1,) * 3, dtype=np.int64)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    wt = w[dx] * w[dy] * w[dz]
                    sl = tuple(slice(R + d - 2 * r, R + d + 2 * r + 1, 2)
                               for d in (dx, dy, dz))
                    child[sl] += wt * ref
        cnt = child
    N = 8 ** k
    return nc, nsc, 100.0 * near * 512 * 512 / N ** 2


# Table 1 (Sect. 4): N_C, N_SC and nf[%] for k = 5..9.
TABLE1 = {5: (3096, 316, 24.41), 6: (166320, 1522, 4.06),
          7: (2640960, 4554, 0.58), 8: (33103296, 9824, 0.077),
          9: (344979432, 32036, 0.010)}


@pytest.mark.parametrize("k", [5, 6, 7, 8, 9])
def test_table1_by_offset_recursion(k):
    nc, nsc, nf = _table1_counts(k)
    NC, NSC, NF = TABLE1[k]
    assert nc == NC and nsc == NSC
    assert round(nf, len(str(NF).split(".")[1])) == NF


@pytest.mark.parametrize("k", [5, 6])
def test_table1_from_points(k):
    P = W.config(f"paper_k{k}")
    plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m)
    s = oracle.structure(plan)
    assert plan.l_hf == k - 4  # Sect. 4 uses l_hf = k - 4
    nc = sum(int(s[f"nc{l}"][0]) for l in range(P.levels + 1))
    nsc = sum(s[f"off{l}"].shape[0] for l in range(P.levels + 1))
    NC, NSC, NF = TABLE1[k]
    assert nc == NC and nsc == NSC
    assert round(100.0 * s["near_entries"][0] / 8 ** (2 * k), 2) == NF
    # at most 27 inadmissible partners per leaf (Sect. 4)
    assert np.bincount(plan.BT.near_t[-1]).max() <= 27


@pytest.mark.parametrize("k", [5, 6])
def test_stored_couplings_pair_by_transposition(k):
    """Every stored coupling (level, o) has its partner (level, -o) stored,
    used by as many blocks, with the antipodal direction, so that
    A_{-o} = A_o^T (the coupling matrix transposes when o and c change sign)
    and half of the bank determines the rest."""
    P = W.config(f"paper_k{k}")
    plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m)
    s = oracle.structure(plan)
    for l in range(P.levels + 1):
        off, cnt = s[f"off{l}"], s[f"offcnt{l}"]
        if not off.shape[0]:
            continue
        index = {tuple(o): i for i, o in enumerate(off)}
        partner = np.array([index[tuple(-o)] for o in off])
        assert np.array_equal(cnt[partner], cnt)
        vec = plan.dirs.vectors(l)
        d = s[f"offdir{l}"]
        assert np.array_equal(vec[d[partner]], -vec[d] + 0.0), l


# ------------------------------------------------------- Alg. 3, dir maps --
def test_direction_counts_and_top_faces():
    D = DirectionSets(3, 5)
    for level in range(6):
        n = D.count(level)
        assert n == (6 * 4 ** (3 - level) if level <= 3 else 1)
        vec = D.vectors(level)
        assert vec.shape == (n, 3)
        if level <= 3:
            assert np.allclose(np.linalg.norm(vec, axis=1), 1.0)
            assert len({tuple(np.round(x, 12)) for x in vec}) == n
    top = D.vectors(3)  # Alg. 3: c_1 = (-1,0,0), c_2 = (1,0,0), c_6 = (0,0,1)
    assert np.array_equal(top, [[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0],
                                [0, 0, -1], [0, 0, 1]])


def _psi_in_face(v, F, j):
    M = max(abs(int(x)) for x in v)
    for d in range(3):
        q = Fraction(int(v[d]), M)
        if not (Fraction(int(F.lo[j, d]), F.den) <= q <= Fraction(int(F.hi[j, d]), F.den)):
            return False
    return True


def test_dir_map_is_lowest_containing_face():
    D = DirectionSets(3, 4)
    rng = np.random.default_rng(2)
    vs = rng.integers(-9, 10, size=(300, 3))
    vs = vs[np.abs(vs).max(axis=1) > 0]
    for level in range(4):
        F = D.faces[level]
        j = D.dir_index(level, vs)
        for v, jj in zip(vs, j):
            inside = [q for q in range(F.axis.shape[0]) if _psi_in_face(v, F, q)]
            assert jj == min(inside)


def test_dir_map_odd_and_cone_bound():
    """dir(-v) = -dir(v); |v/|v| - dir(v)| <= sqrt(2)/n for n sub-faces per
    edge (the cone bound behind (A2), Sect. 2.4)."""
    D = DirectionSets(4, 4)
    r = np.arange(-12, 13)
    v = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    v = v[np.abs(v).max(axis=1) > 0]
    u = v / np.linalg.norm(v, axis=1, keepdims=True)
    for level in range(5):
        vec = D.vectors(level)
        a = D.dir_index(level, v)
        b = D.dir_index(level, -v)
        assert np.allclose(vec[a], -vec[b])
        n = 2 ** (4 - level)
        assert np.max(np.linalg.norm(u - vec[a], axis=1)) <= math.sqrt(2) / n + 1e-12


def test_transfer_direction_is_parent_face():
    D = DirectionSets(3, 4)
    for level in range(3):
        par = D.parent_index(level)
        assert np.array_equal(par, np.arange(D.count(level)) // 4)
    assert np.all(D.parent_index(3) == 0)


def test_active_and_inherited_directions_by_definition():
    P = W.random_problem(21, 300, 250, 40.0, 4, 2)
    plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m)
    assert plan.l_hf >= 1
    # D(t): brute force over all admissible leaves (Def. in Sect. 2.6)
    for tag, D, T, side_idx in (("T", plan.DT, plan.TT, 0), ("S", plan.DS, plan.TS, 1)):
        for level in range(P.levels + 1):
            want = set()
            for t, s in zip(plan.BT.adm_t[level], plan.BT.adm_s[level]):
                m_t = plan.TT.centres(level)[t]
                m_s = plan.TS.centres(level)[s]
                o = np.rint((m_t - m_s) / plan.side(level)).astype(np.int64)
                c = int(plan.dirs.dir_index(level, o))
                want.add((int(t) if side_idx == 0 else int(s), c))
            got = {(int(b), int(c)) for b, c in zip(*np.nonzero(D[level]))}
            assert got == want
    # D^(t): recursive definition
    for level in range(1, P.levels + 1):
        par = plan.TT.parent[level]
        for t in range(plan.TT.keys[level].shape[0]):
            up = plan.DT[level - 1][par[t]] | plan.DhT[level - 1][par[t]]
            want = {int(plan.dirs.dir_index(level, plan.dirs.faces[level - 1].midpoints()[c]))
                    if level <= plan.l_hf else 0 for c in np.flatnonzero(up)}
            assert set(np.flatnonzero(plan.DhT[level][t]).tolist()) == want


def test_high_frequency_level_rule():
    assert oracle.high_frequency_level(20.0, 1.0, 3) == 2
    assert oracle.high_frequency_level(60.0, 1.0, 5) == 4
    assert oracle.high_frequency_level(150.0, 1.0, 7) == 5
    assert oracle.high_frequency_level(400.0, 1.0, 8) == 6
    assert oracle.high_frequency_level(0.0, 1.0, 8) == -1
    for k in range(5, 10):  # Sect. 4: l_hf = k - 4
        assert oracle.high_frequency_level(0.1 * 2.0 ** k, 2.0, k - 3) == k - 4
