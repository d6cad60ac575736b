"""Launch shapes, streamed coupling banks and batched matvecs on the GPU,
against the FP64 oracle (Alg. 4) on the same seeded inputs.

Tolerances as for single plans: plain FP64 1e-12 relative l2, mixed FP32
1e-6; complex64 outputs add their own rounding (2^-24 relative per entry).
Resident-bank FP64 results do not depend on the launch shape at all (every
target's sum over offsets runs in one order; offsets a smaller target
block skips only add exact zeros), so they are compared bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import assert_close, gpu_plan, rel, to_dev

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12
TOL_FP32 = 1e-6

TUNES = [dict(nb=nb, persistent=p, lpt=l, p2p_in_queue=q, compact=0)
         for nb in (64, 32) for p in (1, 0) for l in (1, 0) for q in (0, 1)]
# compacted FP32 columns on every level, for each nb = 64 launch shape
TUNES += [dict(t, compact=2) for t in TUNES if t["nb"] == 64]


_oracle_cache = {}


def oracle_y(P):
    key = (P.name, P.points_T.shape[0], P.points_S.shape[0], P.kappa, P.levels, P.m,
           P.points_T[:1].tobytes(), P.v[:1].tobytes())
    if key not in _oracle_cache:
        _oracle_cache[key] = oracle.matvec(
            oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m), P.v)
    return _oracle_cache[key]


def plan_y(P, precision="fp64", bank_budget=0, tune=None, full_bank=False):
    import torch
    import paper_2004_14229_amd as F
    pt = to_dev(P.points_T)
    ps = to_dev(P.points_S)
    with F.Plan(pt, ps, P.kappa, P.box, P.levels, P.m, precision=precision,
                bank_budget=bank_budget, tune=tune, full_bank=full_bank) as plan:
        y = plan.matvec(to_dev(P.v))
        torch.cuda.synchronize()
        return y.cpu().numpy(), plan.stats()


def small_batch(count=6, seed=41, m=5):
    return W.batch_problems(seed=seed, count=count, m=m, n_lo=400, n_hi=2500)


@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("fp32", TOL_FP32),
                                           ("bf16x3", 2e-5), ("bf16x6", TOL_FP32)])
def test_every_launch_shape_matches_oracle(precision, tol):
    P = W.random_problem(301, 700, 650, 45.0, 4, 3)
    yo = oracle_y(P)
    ys = []
    for t in TUNES:
        y, _ = plan_y(P, precision, tune=t)
        assert_close(y, yo, tol, t)
        ys.append(y)
    if precision == "fp64":
        for y, t in zip(ys[1:], TUNES[1:]):
            assert np.array_equal(y, ys[0]), t


@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("fp32", TOL_FP32)])
def test_streamed_bank_matches_oracle(precision, tol):
    """Bank generated during the matvec, a few matrices at a time, so that
    items are split over many launches (first part stored, later parts
    added)."""
    P = W.random_problem(302, 900, 800, 40.0, 4, 3)
    yo = oracle_y(P)
    y_res, st = plan_y(P, precision)
    K = (P.m + 1) ** 3
    Kp = (K + 31) // 32 * 32
    mat = Kp * Kp * (16 if precision == "fp64" else 8)
    n = st["n_bank_matrices"]
    assert n > 20
    for budget in (mat, 7 * mat, (n // 3) * mat):
        for t in (TUNES[0], TUNES[15], TUNES[-1]):
            y, st2 = plan_y(P, precision, bank_budget=budget, tune=t)
            assert_close(y, yo, tol, (budget, t))
            assert st2["n_couplings"] == st["n_couplings"]
    assert_close(y_res, yo, tol)


@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("fp32", TOL_FP32)])
@pytest.mark.parametrize("m,levels", [(3, 4), (6, 3)])
def test_symmetric_bank_matches_full_bank(precision, tol, m, levels):
    """Resident banks holding one matrix per offset pair (o, -o), the matrix
    of -o applied transposed (Sect. 2.7: A_{-o} = A_o^T), against banks
    holding every matrix and against the oracle, in plain and compacted
    launch shapes.  The bank halves; the results differ by rounding only
    (transposed matrices are summed over k in another order)."""
    P = W.random_problem(321 + m, 1500, 1400, 50.0, levels, m)
    yo = oracle_y(P)
    y_full, st_full = plan_y(P, precision, full_bank=True)
    assert_close(y_full, yo, tol)
    for t in (dict(nb=64, compact=0), dict(nb=64, compact=2), dict(nb=32, persistent=0)):
        y_sym, st_sym = plan_y(P, precision, tune=t)
        assert 2 * st_sym["n_bank_matrices"] == st_full["n_bank_matrices"]
        assert st_sym["n_couplings"] == st_full["n_couplings"]
        assert_close(y_sym, yo, tol, t)
        assert_close(y_sym, y_full, tol, t)


@pytest.mark.parametrize("precision,tol", [("fp32", TOL_FP32), ("bf16x3", 2e-5),
                                           ("bf16x6", TOL_FP32)])
@pytest.mark.parametrize("seed,nt,ns,kappa,levels,m,clustered", [
    (311, 700, 650, 45.0, 4, 3, False), (312, 3000, 2600, 60.0, 5, 3, True),
    (313, 1500, 1400, 30.0, 4, 5, False), (314, 90, 2000, 20.0, 4, 4, False)])
def test_compacted_columns_match_plain(seed, nt, ns, kappa, levels, m, clustered,
                                       precision, tol):
    """Mixed FP32 and BF16 split products with compacted coupling columns
    (on every level, and on the levels the automatic rule picks) against
    the oracle and against the plain items.  Compaction only drops zero
    columns: every target's per-offset sums, FP32 totals and flush points
    are unchanged, so the results agree with the plain items bit for bit."""
    if clustered:
        P = W.clustered_problem(seed, nt, ns, kappa, levels, m)
    else:
        P = W.random_problem(seed, nt, ns, kappa, levels, m)
    yo = oracle_y(P)
    base = dict(nb=64, persistent=1, lpt=1, p2p_in_queue=0)
    y0, st0 = plan_y(P, precision, tune=dict(base, compact=0))
    y1, st1 = plan_y(P, precision, tune=dict(base, compact=1))
    y2, st2 = plan_y(P, precision, tune=dict(base, compact=2))
    for y in (y0, y1, y2):
        assert_close(y, yo, tol)
    assert np.array_equal(y0, y2) and np.array_equal(y0, y1)
    assert st2["m2l_columns"] <= st1["m2l_columns"] <= st0["m2l_columns"]
    assert st1["n_couplings"] == st0["n_couplings"]


@pytest.mark.parametrize("precision,tol", [("fp32", TOL_FP32), ("bf16x3", 2e-5),
                                           ("bf16x6", TOL_FP32)])
def test_compacted_columns_streamed_and_grid(precision, tol):
    """Compacted items split over streamed-bank launches (first part
    stores, later parts add), in grid and persistent launches."""
    P = W.random_problem(315, 1200, 1100, 50.0, 4, 4)
    yo = oracle_y(P)
    K = (P.m + 1) ** 3
    Kp = (K + 31) // 32 * 32
    # FP32: 2 planes x 4 bytes; BF16 split: 4 (x3) or 6 (x6) planes x 2 bytes
    mat = Kp * Kp * (12 if precision == "bf16x6" else 8)
    y_ref, _ = plan_y(P, precision, tune=dict(nb=64, compact=0))
    for pers in (1, 0):
        for budget in (0, 3 * mat):
            y, _ = plan_y(P, precision, bank_budget=budget,
                          tune=dict(nb=64, persistent=pers, compact=2))
            assert_close(y, yo, tol, (pers, budget))
            if budget == 0:
                assert np.array_equal(y, y_ref), pers


def test_streamed_bank_uniform2k_fp32():
    P = W.config("uniform2k")
    yo = oracle_y(P)
    y, st = plan_y(P, "fp32", bank_budget=50 * 128 * 128 * 8)
    assert_close(y, yo, TOL_FP32)


def _batch_vectors(probs, c64):
    import torch
    dt = np.complex64 if c64 else np.complex128
    return [torch.from_numpy(P.v.astype(dt)).cuda() for P in probs]


def _batch_check(probs, ys, tol, c64):
    for P, y in zip(probs, ys):
        yo = oracle_y(P)
        yy = y.cpu().numpy().astype(np.complex128)
        assert_close(yy, yo, tol + (1e-7 if c64 else 0.0), P.name)


@pytest.mark.parametrize("precision,tol,c64,budget", [
    ("fp64", TOL_FP64, False, 0), ("fp32", TOL_FP32, True, 0),
    ("fp32", TOL_FP32, True, 1), ("fp64", TOL_FP64, False, 1)])
def test_batch_matches_oracle(precision, tol, c64, budget):
    """Small batch of uneven uniform and clustered problems (the batched
    workload's generator at small N); budget 1: streamed banks, generated
    into the batch's workspace (a third of their total) over several
    launches."""
    import torch
    import paper_2004_14229_amd as F
    probs = small_batch()
    K = (probs[0].m + 1) ** 3
    Kp = (K + 31) // 32 * 32
    mat = Kp * Kp * (16 if precision == "fp64" else 8)
    plans = [gpu_plan(P, precision) if not budget else
             F.Plan(to_dev(P.points_T), to_dev(P.points_S), P.kappa, P.box, P.levels, P.m,
                    precision=precision, bank_budget=mat)
             for P in probs]
    ws = 0
    if budget:
        total = sum(p.stats()["n_bank_matrices"] for p in plans)
        ws = max(1, total // 3) * mat
    with F.Batch(plans, workspace_bytes=ws) as b:
        ys = b.matvec(_batch_vectors(probs, c64))
        torch.cuda.synchronize()
        _batch_check(probs, ys, tol, c64)
    for p in plans:
        p.close()


def test_batch_graph_replays_match_eager():
    """The batched matvec captured in a HIP graph and replayed several
    times, with eager work and synchronisations between replays; every
    replay equals the eager (uncaptured) result bit for bit."""
    import torch
    import paper_2004_14229_amd as F
    probs = small_batch(count=5, seed=43)
    plans = [gpu_plan(P, "fp32") for P in probs]
    s = torch.cuda.Stream()
    with F.Batch(plans) as b:
        vs = _batch_vectors(probs, True)
        torch.cuda.synchronize()
        b.set_graph(False)
        with torch.cuda.stream(s):
            eager = [y.clone() for y in b.matvec(vs, stream=s)]
        s.synchronize()
        b.set_graph(True)
        outs = [torch.empty_like(y) for y in eager]
        for r in range(4):
            with torch.cuda.stream(s):
                for y in outs:
                    y.fill_(float("nan"))
                b.matvec(vs, outs, stream=s)
            s.synchronize()
            extra = torch.randn(1000, device="cuda").sum()  # eager work between replays
            torch.cuda.synchronize()
            assert torch.isfinite(extra)
            for y, e in zip(outs, eager):
                assert torch.equal(y, e), r
        _batch_check(probs, outs, TOL_FP32, True)
    for p in plans:
        p.close()


def test_batch_with_empty_problems():
    import torch
    import paper_2004_14229_amd as F
    probs = small_batch(count=3, seed=44)
    probs.append(W.random_problem(45, 50, 0, 10.0, 3, 5))
    probs.append(W.random_problem(46, 0, 40, 10.0, 3, 5))
    plans = [gpu_plan(P, "fp64") for P in probs]
    with F.Batch(plans) as b:
        ys = b.matvec(_batch_vectors(probs, False))
        torch.cuda.synchronize()
        for P, y in zip(probs[:3], ys[:3]):
            assert_close(y.cpu().numpy(), oracle_y(P), TOL_FP64)
        assert ys[3].shape == (50,) and torch.all(ys[3] == 0)
        assert ys[4].shape == (0,)
    for p in plans:
        p.close()


def test_plan_in_batch_cannot_be_destroyed_or_retuned():
    import paper_2004_14229_amd as F
    probs = small_batch(count=2, seed=47)
    plans = [gpu_plan(P, "fp64") for P in probs]
    b = F.Batch(plans)
    with pytest.raises(F.FdmError):
        plans[0].set_tune({"nb": 32})
    with pytest.raises(F.FdmError):
        plans[0].close()
    b.close()
    plans[0].set_tune({"nb": 32})
    for p in plans:
        p.close()


def test_autotune_plan_and_batch():
    """The autotuner times every candidate, keeps the fastest, and the
    tuned plan / batch still matches the oracle."""
    import torch
    import paper_2004_14229_amd as F
    P = W.random_problem(303, 800, 760, 35.0, 4, 3)
    yo = oracle_y(P)
    plan = gpu_plan(P, "fp32")
    best, ms, y = plan.autotune(to_dev(P.v))
    torch.cuda.synchronize()
    assert len(ms) == 8 and all(t > 0 for t in ms)
    assert best == plan.get_tune()
    assert_close(y.cpu().numpy(), yo, TOL_FP32)
    y2 = plan.matvec(to_dev(P.v))
    torch.cuda.synchronize()
    assert_close(y2.cpu().numpy(), yo, TOL_FP32)
    # the two other compaction modes as candidates 9 and 10
    best, ms, y = plan.autotune(to_dev(P.v), max_candidates=10)
    torch.cuda.synchronize()
    assert len(ms) == 10 and all(t > 0 for t in ms)
    assert best == plan.get_tune()
    y3 = plan.matvec(to_dev(P.v))
    torch.cuda.synchronize()
    assert_close(y3.cpu().numpy(), yo, TOL_FP32)
    plan.close()

    probs = small_batch(count=4, seed=48)
    plans = [gpu_plan(Q, "fp32") for Q in probs]
    with F.Batch(plans) as b:
        vs = _batch_vectors(probs, True)
        best, ms, ys = b.autotune(vs)
        torch.cuda.synchronize()
        assert len(ms) == 4 and all(t > 0 for t in ms)
        assert best == b.get_tune() and best["persistent"] == 1
        _batch_check(probs, ys, TOL_FP32, True)
        ys = b.matvec(vs)
        torch.cuda.synchronize()
        _batch_check(probs, ys, TOL_FP32, True)
        best, ms, ys = b.autotune(vs, max_candidates=6)
        torch.cuda.synchronize()
        assert len(ms) == 6 and all(t > 0 for t in ms)
        assert best == b.get_tune()
        ys = b.matvec(vs)
        torch.cuda.synchronize()
        _batch_check(probs, ys, TOL_FP32, True)
    for p in plans:
        p.close()
