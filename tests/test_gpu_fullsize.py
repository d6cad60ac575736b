"""Full-size parity: the HIP library at the benchmark workloads against the
FP64 oracle's Alg. 4 on stored sampled rows (tests/golden/*_rows.npz, written
by tests/golden/make_golden.py from the oracle alone).

Tolerances: plain FP64 1e-12 relative l2 over the sampled rows; mixed FP32
1e-6 (the stated bound of the mixed path); BF16 split products within 3x the
error of the oracle's emulation of that arithmetic on the same rows.  Each
bound holds for the relative l2 error and for every sampled entry against
the largest reference entry.  (The full FP32 vector is also compared with
the plain FP64 GPU vector: a consistency check over every row, not parity.)
The batched workload (64 problems, complex64 in and out, mixed FP32): 1e-6
plus the complex64 rounding of y (1e-7) on the stored rows of four problems.

Rows: 64 seeded rows at N = 1e5; 256 seeded rows plus the targets nearest
the box corners, face centres and centre at N = 1e6 (boundary leaves and
interior leaves), at N = 4e6 (32 + 15) and on the paper's k = 6 grid
(256 + 15).  The 4e6-point workload runs with its bank streamed through a
24 GB workspace where the bank does not fit beside its moments (FP64, BF16
splits; the symmetric FP32 bank of 99 GB is resident);
of its runs only the BF16 three-product one is in the default suite.
"""
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import assert_close, gpu_plan, rel, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_cache = {}


BUDGET = {"uniform4m": 24 << 30}
RESIDENT = {("uniform4m", "fp32")}  # its symmetric FP32 bank (99 GB) fits

# The 4e6-point runs take one to three minutes each (the bank is regenerated
# every matvec); the BF16 three-product one always runs, the others when
# FDM_LARGE_TESTS=1.
large = pytest.mark.skipif(os.environ.get("FDM_LARGE_TESTS") != "1",
                           reason="4e6-point run of minutes: set FDM_LARGE_TESTS=1")


def run(name, prec, aca_eps=0.0):
    import torch
    import paper_2004_14229_amd as F
    key = (name, prec, aca_eps)
    if key not in _cache:
        P = W.config(name)
        print(f"fullsize {name} {prec} aca_eps={aca_eps}", flush=True)
        pt = to_dev(P.points_T)
        ps = pt if P.same_points else to_dev(P.points_S)
        with F.Plan(pt, ps, P.kappa, P.box, P.levels, P.m, precision=prec,
                    bank_budget=0 if aca_eps or (name, prec) in RESIDENT
                    else BUDGET.get(name, 0),
                    aca_eps=aca_eps) as plan:  # (low-rank banks stay resident)
            y = plan.matvec(to_dev(P.v))
            torch.cuda.synchronize()
            _cache[key] = (y.cpu().numpy(), plan.stats())
        del y
        torch.cuda.empty_cache()
    return _cache[key]


def golden(name, key="y"):
    path = os.path.join(GOLDEN, f"{name}_rows.npz")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle rows {path} (tests/golden/make_golden.py {name})")
    g = np.load(path)
    return g["rows"], g[key]


@pytest.mark.parametrize("name", ["uniform100k", "uniform1m", "paper_k6"])
def test_fp64_sampled_rows(name):
    rows, yo = golden(name)
    y, st = run(name, "fp64")
    assert_close(y[rows], yo, 1e-12)
    assert np.all(np.isfinite(y))
    if name == "paper_k6":  # Table 1, k = 6
        assert st["n_couplings"] == 166320 and st["n_stored_couplings"] == 1522
        assert round(100.0 * st["near_entries"] / 8 ** 12, 2) == 4.06
        _cache.pop((name, "fp64", 0.0), None)


@pytest.mark.parametrize("name", ["uniform100k", "uniform1m"])
def test_fp32_sampled_rows_and_full_vector(name):
    rows, yo = golden(name)
    y32, st = run(name, "fp32")
    assert_close(y32[rows], yo, 1e-6)
    y64, _ = run(name, "fp64")
    assert_close(y32, y64, 1e-6)  # consistency over every row (GPU vs GPU)
    _cache.pop((name, "fp64", 0.0), None)


@pytest.mark.parametrize("name", ["uniform100k", "uniform1m"])
def test_bf16x3_sampled_rows(name):
    rows, yo = golden(name)
    _, ye = golden(name, "y_bf16x3")
    y, st = run(name, "bf16x3")
    _cache.pop((name, "bf16x3", 0.0), None)
    assert np.all(np.isfinite(y))
    assert_close(y[rows], yo, 3 * rel(ye, yo))


@pytest.mark.parametrize("name", ["uniform100k", "uniform1m"])
def test_bf16x6_sampled_rows(name):
    """Six-product BF16 split: the mixed-precision bound 1e-6 and within 3x
    of the oracle's emulation of the split arithmetic on the same rows."""
    rows, yo = golden(name)
    _, ye = golden(name, "y_bf16x6")
    y, st = run(name, "bf16x6")
    _cache.pop((name, "bf16x6", 0.0), None)
    assert np.all(np.isfinite(y))
    assert_close(y[rows], yo, min(1e-6, 3 * rel(ye, yo)))


@pytest.mark.parametrize("name", ["uniform100k", "uniform1m",
                                  pytest.param("uniform4m", marks=large)])
def test_aca_sampled_rows(name):
    """Low-rank couplings (ACA to 1e-7, FP32 matrix-core stages) against the
    oracle's dense-coupling rows: the mixed-precision bound 1e-6 covers the
    compression and the FP32 arithmetic together."""
    rows, yo = golden(name)
    y, st = run(name, "fp32", 1e-7)
    _cache.pop((name, "fp32", 1e-7), None)
    assert np.all(np.isfinite(y))
    assert 0 < st["aca_flops"] <= st["aca_issued_flops"]
    assert_close(y[rows], yo, 1e-6)


def test_structure_paper_grid_k6():
    """Table 1's k = 6 row from the GPU's structure, and the trees, block
    partition and direction sets bit for bit against the oracle's."""
    import oracle
    from test_gpu_parity import check_structure
    P = W.config("paper_k6")
    with gpu_plan(P) as gp:
        check_structure(P, gp, oracle.build(P.points_T, P.points_S, P.kappa, P.box,
                                             P.levels, P.m))


@pytest.mark.parametrize("prec", [pytest.param("fp32", marks=large), "bf16x3",
                                  pytest.param("bf16x6", marks=large)])
def test_uniform4m_sampled_rows(prec):
    """4e6 points, kappa = 400, 8 levels, m = 6 (the large high-frequency
    workload), FP32 with its symmetric bank resident (99 GB), the BF16 splits
    with theirs streamed: FP32 within 1e-6 of the oracle's rows, BF16
    split products within 3x the oracle's emulation of them (and the
    six-product split within 1e-6 too)."""
    rows, yo = golden("uniform4m")
    y, st = run("uniform4m", prec)
    _cache.pop(("uniform4m", prec, 0.0), None)
    assert np.all(np.isfinite(y))
    assert st["n_stored_couplings"] == 200258
    if prec == "fp32":  # resident: one matrix per offset pair
        assert st["n_bank_matrices"] == 200258 // 2
    tol = 1e-6 if prec == "fp32" else 3 * rel(golden("uniform4m", f"y_{prec}")[1], yo)
    if prec == "bf16x6":
        tol = min(tol, 1e-6)
    assert_close(y[rows], yo, tol)


def test_batched_workload_sampled_rows():
    """The 64-problem batched workload as the benchmark runs it: mixed FP32,
    banks generated into the batch workspace, one device queue, graph
    replay on a side stream."""
    import torch
    import paper_2004_14229_amd as F
    g = np.load(os.path.join(GOLDEN, "batch_rows.npz"))
    probs = W.batch_problems()
    plans = [F.Plan(to_dev(Q.points_T), to_dev(Q.points_S), Q.kappa, Q.box, Q.levels, Q.m,
                    precision="fp32", bank_budget=1 << 30) for Q in probs]
    try:
        with F.Batch(plans) as b:
            vs = [torch.from_numpy(Q.v.astype(np.complex64)).cuda() for Q in probs]
            torch.cuda.synchronize()
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                ys = b.matvec(vs, stream=s)
                ys2 = b.matvec(vs, [torch.empty_like(y) for y in ys], stream=s)
            s.synchronize()
            checked = 0
            for key in g.files:
                if not key.startswith("rows"):
                    continue
                i = int(key[4:])
                for out in (ys, ys2):
                    yy = out[i].cpu().numpy().astype(np.complex128)[g[key]]
                    assert_close(yy, g[f"y{i}"], 1e-6 + 1e-7, i)
                checked += 1
            assert checked == 4
            for y in ys:
                assert torch.isfinite(torch.view_as_real(y)).all()
    finally:
        for p in plans:
            p.close()
