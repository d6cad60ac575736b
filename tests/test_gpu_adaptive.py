"""Adaptive trees on the GPU (Alg. 1's n_max stop rule; Alg. 2 with leaves
on several levels; Alg. 4 with S2M / L2T at the leaves of every level and
near-field blocks on every level), through the C ABI, against the oracle
built with the same n_max.

Tolerances as for uniform trees: structure bit for bit (boxes that exist,
block counts and offsets per level, direction sets, near-field pair and
entry counts); plain FP64 1e-12; mixed FP32 1e-6; the six-product BF16 split
within the mixed bound and 4x of the oracle's emulation."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import assert_close, rel, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (seed, n_T, n_S, kappa, levels, m, n_max)
    "clustered": (501, 1500, 1400, 25.0, 6, 3, 8),
    "clustered_hf": (502, 2000, 1800, 60.0, 6, 3, 24),
    "uniform": (503, 1200, 1000, 15.0, 5, 4, 4),
    "tiny_leaves": (504, 700, 650, 10.0, 5, 2, 1),
}


def problem(name):
    seed, nT, nS, kappa, levels, m, n_max = CASES[name]
    if name.startswith("uniform"):
        P = W.random_problem(seed, nT, nS, kappa, levels, m)
    else:
        P = W.clustered_problem(seed, nT, nS, kappa, levels, m)
    return P, n_max


def plan(P, n_max, precision="fp64", **kw):
    import paper_2004_14229_amd as F
    return F.Plan(to_dev(P.points_T), to_dev(P.points_S), P.kappa, P.box, P.levels, P.m,
                  precision=precision, n_max=n_max, **kw)


def oracle_plan(P, n_max):
    return oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m, n_max=n_max)


def matvec(gp, P):
    import torch
    y = gp.matvec(to_dev(P.v))
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("name", sorted(CASES))
def test_structure_bit_exact(name):
    from test_gpu_parity import check_structure
    P, n_max = problem(name)
    op = oracle_plan(P, n_max)
    # the case really is adaptive: leaves and near-field blocks on 2+ levels
    assert len([l for l in range(P.levels + 1) if op.TT.is_leaf(l).any()]) >= 2
    assert len([l for l in range(P.levels + 1) if op.BT.near_t[l].size]) >= 2
    with plan(P, n_max) as gp:
        check_structure(P, gp, op)
        st = gp.stats()
        assert st["n_couplings"] == op.BT.n_admissible()


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp64_and_fp32_match_oracle(name):
    P, n_max = problem(name)
    yo = oracle.matvec(oracle_plan(P, n_max), P.v)
    with plan(P, n_max, "fp64") as gp:
        y64 = matvec(gp, P)
    assert_close(y64, yo, 1e-12, f"{name} fp64")
    with plan(P, n_max, "fp32") as gp:
        y32 = matvec(gp, P)
    assert_close(y32, yo, 1e-6, f"{name} fp32")


def test_bf16x6_matches_emulation():
    P, n_max = problem("clustered")
    yo, ye = oracle.matvec(oracle_plan(P, n_max), P.v, m2l=("fp64", "bf16x6"))
    with plan(P, n_max, "bf16x6") as gp:
        y = matvec(gp, P)
    assert_close(y, yo, min(1e-6, 4 * rel(ye, yo)))


def test_single_leaf_is_the_dense_product():
    """n_max >= N: the root is the only leaf, all of A is one near-field
    block."""
    P, _ = problem("tiny_leaves")
    n = max(P.points_T.shape[0], P.points_S.shape[0])
    with plan(P, n) as gp:
        y = matvec(gp, P)
        assert gp.stats()["n_couplings"] == 0
    yd = oracle.dense_matvec(P.points_T, P.points_S, P.v, P.kappa)
    assert_close(y, yd, 1e-12)


def test_streamed_bank_launch_shapes_and_low_rank():
    """Adaptive plans with the bank generated a few matrices at a time, with
    the grid launch and 32-target items, and with low-rank couplings."""
    P, n_max = problem("clustered_hf")
    op = oracle_plan(P, n_max)
    yo = oracle.matvec(op, P.v)
    with plan(P, n_max, "fp32", bank_budget=3 * 2 * 4 * 64 * 64) as gp:
        y1 = matvec(gp, P)
        gp.set_tune({"nb": 32, "persistent": 0, "lpt": 0, "compact": 0, "p2p_in_queue": 1})
        y2 = matvec(gp, P)
    assert_close(y1, yo, 1e-6)
    assert_close(y2, yo, 1e-6)
    ya = oracle.matvec(op, P.v, m2l="aca:1e-7")
    with plan(P, n_max, "fp32", aca_eps=1e-7) as gp:
        y3 = matvec(gp, P)
    assert_close(y3, ya, 1e-6)


def test_batch_of_adaptive_and_uniform_plans():
    """A batch mixing an adaptive plan and a uniform one (the near field of
    the adaptive plan runs as its own launch, the uniform one's queued)."""
    import torch
    import paper_2004_14229_amd as F
    P1, n1 = problem("clustered")
    P2, _ = problem("uniform")
    P2 = W.random_problem(505, 900, 800, 15.0, 5, 3)
    plans = [plan(P1, n1, "fp32"), plan(P2, 0, "fp32")]
    try:
        with F.Batch(plans) as b:
            ys = b.matvec([to_dev(P1.v), to_dev(P2.v)])
            torch.cuda.synchronize()
            y1, y2 = (y.cpu().numpy() for y in ys)
    finally:
        for p in plans:
            p.close()
    assert_close(y1, oracle.matvec(oracle_plan(P1, n1), P1.v), 1e-6)
    assert_close(y2, oracle.matvec(oracle_plan(P2, None), P2.v), 1e-6)


def test_near_field_items_span_chunks_and_range_batches():
    """A clump of 1500 targets inside one box of level 3 against sparse
    uniform sources, whose level-3 boxes are leaves (n_max = 8): that target
    box meets 418 source leaves at its level's inadmissible offsets.  Its
    near-field work is six items of at most 256 points, each with two
    batches of at most 256 source ranges (the layout of the adaptive
    near-field kernel).  Structure bit for bit, FP64 and FP32 against the
    oracle."""
    from test_gpu_parity import check_structure
    rng = np.random.default_rng(505)
    PT = 0.26 + 0.1 * rng.random((1500, 3))
    PS = W.unit_cube_points(rng, 2000)
    P = W.Problem("clump_vs_sparse", PT, PS, W.complex_normal(rng, 2000), 60.0,
                  (0.0, 0.0, 0.0, 1.0, 1.0, 1.0), 5, 3)
    n_max = 8
    op = oracle_plan(P, n_max)
    nt = op.BT.near_t[3]
    per_box = np.bincount(nt, minlength=len(op.TT.count[3]))
    b = int(np.argmax(per_box))
    assert per_box[b] > 256 and op.TT.count[3][b] > 256  # several items, several batches
    yo = oracle.matvec(op, P.v)
    with plan(P, n_max, "fp64") as gp:
        check_structure(P, gp, op)
        y64 = matvec(gp, P)
    assert_close(y64, yo, 1e-12, "fp64")
    with plan(P, n_max, "fp32") as gp:
        y32 = matvec(gp, P)
    assert_close(y32, yo, 1e-6, "fp32")
