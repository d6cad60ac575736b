"""Non-cubic root boxes on the GPU (Sect. 2.1: any axis-parallel box), through
the C ABI, against the oracle: structure bit for bit (block offsets,
directions evaluated exactly on the centre offsets o * h), plain FP64 within
1e-12, mixed FP32 within 1e-6, the six-product BF16 split within the mixed
bound; also with adaptive trees and a streamed bank."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import assert_close, rel, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    # name: (seed, n_T, n_S, kappa, box, levels, m, n_max)
    "flat": (601, 1200, 1100, 20.0, (0.0, -0.5, 0.25, 2.0, 0.5, 0.75), 4, 3, 0),
    "long_hf": (602, 1500, 1400, 40.0, (-1.0, 0.0, 0.0, 3.0, 1.0, 1.0), 5, 3, 0),
    "tenths": (603, 900, 800, 15.0, (0.1, 0.2, 0.3, 0.8, 0.9, 1.3), 4, 4, 0),
    "adaptive": (604, 1400, 1300, 25.0, (0.0, 0.0, 0.0, 1.5, 1.0, 0.75), 5, 3, 6),
}


def problem(name):
    seed, nT, nS, kappa, box, levels, m, n_max = CASES[name]
    return W.random_problem(seed, nT, nS, kappa, levels, m, box), n_max


def plan(P, n_max, precision="fp64", **kw):
    import paper_2004_14229_amd as F
    return F.Plan(to_dev(P.points_T), to_dev(P.points_S), P.kappa, P.box, P.levels, P.m,
                  precision=precision, n_max=n_max, **kw)


def oracle_plan(P, n_max):
    return oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m,
                        n_max=n_max or None)


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
    assert op.l_hf >= 1 and op.BT.n_admissible() > 0
    with plan(P, n_max) as gp:
        check_structure(P, gp, op)


@pytest.mark.parametrize("name", sorted(CASES))
def test_matches_oracle(name):
    P, n_max = problem(name)
    op = oracle_plan(P, n_max)
    yo, ye = oracle.matvec(op, P.v, m2l=("fp64", "bf16x6"))
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-6), ("bf16x6", min(1e-6, 4 * rel(ye, yo)))):
        with plan(P, n_max, prec) as gp:
            y = matvec(gp, P)
        assert_close(y, yo, tol, f"{name} {prec}")


def test_streamed_bank():
    P, n_max = problem("long_hf")
    yo = oracle.matvec(oracle_plan(P, n_max), P.v)
    with plan(P, n_max, "fp32", bank_budget=4 * 64 * 64 * 2 * 4) as gp:
        y = matvec(gp, P)
    assert_close(y, yo, 1e-6)
