"""Several right-hand sides on one plan (fdm_plan_matvec_multi): each result
bit for bit that of fdm_plan_matvec on the same vector (the near field
evaluates each kernel value once for up to four vectors but sums in the same
order), for uniform, adaptive, low-rank, streamed-bank and paper-grid plans,
complex128 and complex64, and within the usual bounds of the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import assert_close, to_dev

pytestmark = pytest.mark.gpu


def vectors(n, nrhs, seed):
    rng = np.random.default_rng(seed)
    return np.stack([W.complex_normal(rng, n) for _ in range(nrhs)])


def check(plan, V, c64=False):
    import torch
    dt = torch.complex64 if c64 else torch.complex128
    Vd = torch.from_numpy(V).to(dt).cuda()
    Y = plan.matvec_multi(Vd)
    torch.cuda.synchronize()
    for r in range(V.shape[0]):
        y = plan.matvec(Vd[r].clone())
        torch.cuda.synchronize()
        d = (Y[r] - y).abs().max().item() / max(y.abs().max().item(), 1e-300)
        assert torch.equal(Y[r], y), (r, d)
    return Y.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uniform_plan(prec):
    import paper_2004_14229_amd as F
    P = W.random_problem(701, 900, 850, 25.0, 4, 3)
    V = vectors(P.points_S.shape[0], 5, 1)  # a pass of four and a pass of one
    with F.Plan(to_dev(P.points_T), to_dev(P.points_S), P.kappa, P.box, P.levels, P.m,
                precision=prec) as plan:
        Y = check(plan, V)
        check(plan, V[:2], c64=True)
    op = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m)
    for r in (0, 4):
        assert_close(Y[r], oracle.matvec(op, V[r]), 1e-12 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("kind", ["adaptive", "aca", "streamed", "queued_near_field"])
def test_other_plans(kind):
    import paper_2004_14229_amd as F
    P = W.clustered_problem(702, 1000, 900, 20.0, 5, 3)
    kw = {"adaptive": dict(n_max=8), "aca": dict(aca_eps=1e-7),
          "streamed": dict(bank_budget=6 * 64 * 64 * 8), "queued_near_field": {}}[kind]
    with F.Plan(to_dev(P.points_T), to_dev(P.points_S), P.kappa, P.box, P.levels, P.m,
                precision="fp32", **kw) as plan:
        if kind == "queued_near_field":
            plan.set_tune({"p2p_in_queue": 1})
        check(plan, vectors(P.points_S.shape[0], 3, 2))


def test_paper_grid_near_field_reuse():
    """Sect. 4's k = 5 grid (512 points per leaf: the near field dominates):
    four right-hand sides in one call against four calls; the kernel values
    are evaluated once per pair for all four (timings printed)."""
    import time
    import torch
    import paper_2004_14229_amd as F
    P = W.config("paper_k5")
    V = vectors(P.points_S.shape[0], 4, 3)
    pt = to_dev(P.points_T)
    with F.Plan(pt, pt, P.kappa, P.box, P.levels, P.m, precision="fp64") as plan:
        check(plan, V)
        Vd = torch.from_numpy(V).cuda()
        Y = plan.matvec_multi(Vd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.matvec_multi(Vd, Y)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for r in range(4):
            plan.matvec(Vd[r], Y[r])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    print(f"paper_k5, 4 vectors: one call {1e3 * (t1 - t0):.1f} ms, four calls "
          f"{1e3 * (t2 - t1):.1f} ms")


def test_invalid_arguments():
    import ctypes
    import torch
    import paper_2004_14229_amd as F
    P = W.random_problem(703, 100, 90, 5.0, 2, 2)
    with F.Plan(to_dev(P.points_T), to_dev(P.points_S), P.kappa, P.box, P.levels, P.m) as plan:
        V = torch.zeros(2, 90, dtype=torch.complex128, device="cuda")
        Y = torch.zeros(2, 100, dtype=torch.complex128, device="cuda")
        L = F.lib()
        assert L.fdm_plan_matvec_multi(plan._h, V.data_ptr(), Y.data_ptr(), 0, 0, None) == -1
        assert L.fdm_plan_matvec_multi(plan._h, V.data_ptr(), Y.data_ptr(), 2, 2, None) == -1
        assert L.fdm_plan_matvec_multi(plan._h, V.data_ptr(), V.data_ptr(), 2, 0, None) == -1
        assert L.fdm_plan_matvec_multi(None, V.data_ptr(), Y.data_ptr(), 2, 0, None) == -1
        torch.cuda.synchronize()
