"""The allocation-free matvec (fdm_plan_matvec_noalloc) against the plan's
ordinary matvec (fdm_plan_matvec / _c64) on the same plans, through the C ABI:
two plans in a row, the second smaller, each run twice through the static
workspace (so the second call finds the first call's matrices there), in
plain FP64 and mixed FP32, complex128 and complex64.  The two entry points
run the same kernels on the same launches, so results agree bit for bit;
the FP64 result is also checked against the oracle (1e-12 relative l2).
Also: the argument and state errors of the entry point."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import assert_close, rel, to_dev

pytestmark = pytest.mark.gpu

MATRIX_BYTES = {"fp64": 2 * 128 * 128 * 8, "fp32": 2 * 128 * 128 * 4}  # m = 4: Kp = 128


def _plan(P, precision, budget):
    import paper_2004_14229_amd as F
    return F.Plan(to_dev(P.points_T), to_dev(P.points_S), P.kappa, P.box, P.levels, P.m,
                  precision=precision, bank_budget=budget)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_matvec_two_calls(precision):
    import torch
    cases = [W.random_problem(901, 2600, 2400, 24.0, 3, 4),
             W.random_problem(902, 1100, 900, 18.0, 3, 4)]  # second call: smaller input
    for P in cases:
        print(f"noalloc {precision}: n_T={P.points_T.shape[0]} n_S={P.points_S.shape[0]}",
              flush=True)
        with _plan(P, precision, 7 * MATRIX_BYTES[precision]) as plan:
            plan.prepare()
            assert plan.coupling_launches() > 1  # many bank ranges through the workspace
            for dtype in (torch.complex128, torch.complex64):
                v = to_dev(P.v).to(dtype)
                y_ref = plan.matvec(v)
                y_na = torch.full_like(y_ref, float("nan"))
                plan.matvec_noalloc(v, y_na)
                torch.cuda.synchronize()
                assert torch.equal(y_na, y_ref)
                y_na.fill_(float("nan"))
                plan.matvec_noalloc(v, y_na)
                torch.cuda.synchronize()
                assert torch.equal(y_na, y_ref)
            if precision == "fp64":
                yo = oracle.matvec(oracle.build(P.points_T, P.points_S, P.kappa, P.box,
                                                P.levels, P.m), P.v)
                y = plan.matvec(to_dev(P.v)).cpu().numpy()
                assert_close(y, yo, 1e-12)


def test_noalloc_rejects_what_it_cannot_run():
    import torch
    import paper_2004_14229_amd as F
    L = F.lib()
    P = W.random_problem(903, 900, 800, 20.0, 3, 4)
    v = to_dev(P.v)
    y = torch.empty(P.points_T.shape[0], dtype=torch.complex128, device=v.device)
    # resident bank: the ordinary matvec allocates nothing already
    with _plan(P, "fp64", 0) as plan:
        plan.prepare()
        assert L.fdm_plan_matvec_noalloc(plan._h, F.fdm._ptr(v), F.fdm._ptr(y), 0, None) == -1
    # workspace beyond the static 64 MiB (FP64 m = 4: 262 KiB per matrix)
    with _plan(P, "fp64", 300 * MATRIX_BYTES["fp64"]) as plan:
        plan.prepare()
        st = L.fdm_plan_matvec_noalloc(plan._h, F.fdm._ptr(v), F.fdm._ptr(y), 0, None)
        msg = L.fdm_last_error()
        ws = min(plan.stats()["n_bank_matrices"], 300) * MATRIX_BYTES["fp64"]
        assert st == (-1 if ws > 64 << 20 else 0)
        assert st == 0 or b"static workspace" in msg
    # not prepared: the schedule would have to be allocated
    with _plan(P, "fp64", 4 * MATRIX_BYTES["fp64"]) as plan:
        st = L.fdm_plan_matvec_noalloc(plan._h, F.fdm._ptr(v), F.fdm._ptr(y), 0, None)
        assert st == -6
        plan.prepare()
        assert L.fdm_plan_matvec_noalloc(plan._h, F.fdm._ptr(v), F.fdm._ptr(y), 2, None) == -1
        assert L.fdm_plan_matvec_noalloc(plan._h, F.fdm._ptr(v), F.fdm._ptr(y), 0, None) == 0
    assert L.fdm_plan_matvec_noalloc(None, None, None, 0, None) == -1
    torch.cuda.synchronize()
