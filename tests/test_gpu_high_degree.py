"""Interpolation degrees m = 7 and 8 (K = 512 and 729 nodes per box): the
coupling matrices have more rows than one workgroup's waves cover, so every
coupling item runs once per row block (256 or 384 rows each).  Against the
oracle's Alg. 4 on every target row, stored by tests/golden/make_golden.py
(the oracle takes minutes at these degrees).

Tolerances as for the other degrees: plain FP64 1e-12; mixed FP32 1e-6; BF16
split products within 4x of the oracle's emulation of the same arithmetic
(and the six-product split within 1e-6 as well).  The structure (trees,
block partition, directions) bit for bit against the oracle's."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import assert_close, gpu_matvec, gpu_plan, rel, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    path = os.path.join(GOLDEN, f"{name}_rows.npz")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle rows {path} (tests/golden/make_golden.py {name})")
    return np.load(path)


@pytest.mark.parametrize("name", ["degree7", "degree8"])
def test_structure_bit_exact(name):
    from test_gpu_parity import check_structure
    P = W.config(name)
    with gpu_plan(P) as gp:
        check_structure(P, gp, oracle.build(P.points_T, P.points_S, P.kappa, P.box,
                                             P.levels, P.m))
        st = gp.stats()
        assert st["K"] == (P.m + 1) ** 3 and st["n_couplings"] > 0


@pytest.mark.parametrize("name", ["degree7", "degree8"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_matches_oracle(name, prec):
    g = golden(name)
    P = W.config(name)
    assert np.array_equal(g["rows"], np.arange(P.points_T.shape[0]))
    y, _ = gpu_matvec(P, prec)
    yo = g["y"]
    assert np.all(np.isfinite(y))
    if prec == "fp64":
        tol = 1e-12
    elif prec == "fp32":
        tol = 1e-6
    else:
        emulated = rel(g[f"y_{prec}"], yo)
        assert emulated > 0
        tol = 4 * emulated if prec == "bf16x3" else min(1e-6, 4 * emulated)
    assert_close(y, yo, tol, f"{name} {prec}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_streamed_bank_and_launch_shapes(prec):
    """m = 8 with the bank generated a few matrices at a time (items split
    into parts that add to the result), and the grid launch with 32-target
    items: the same bound against the oracle."""
    import torch
    import paper_2004_14229_amd as F
    g = golden("degree8")
    P = W.config("degree8")
    K = (P.m + 1) ** 3
    mat = (K + 31) // 32 * 32
    mat = mat * mat * 2 * (8 if prec == "fp64" else 4)
    with F.Plan(to_dev(P.points_T), to_dev(P.points_S), P.kappa, P.box, P.levels, P.m,
                precision=prec, bank_budget=5 * mat) as plan:
        y1 = plan.matvec(to_dev(P.v)).cpu().numpy()
        plan.set_tune({"nb": 32, "persistent": 0, "lpt": 0, "compact": 0, "p2p_in_queue": 0})
        y2 = plan.matvec(to_dev(P.v)).cpu().numpy()
        torch.cuda.synchronize()
        assert plan.coupling_launches() > 4
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert_close(y1, g["y"], tol)
    assert_close(y2, g["y"], tol)
