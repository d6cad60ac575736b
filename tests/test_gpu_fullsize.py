"""Full-size parity: the HIP library at the benchmark workloads against the
FP64 oracle's Alg. 4 on stored sampled rows (tests/golden/*_rows.npz, written
by tests/golden/make_golden.py from the oracle alone).

Tolerances: plain FP64 1e-12 relative l2 over the sampled rows; mixed FP32
1e-6 (the stated bound of the mixed path); the FP32 result also against the
plain GPU result on the full vector; BF16 split products within 3x the
error of the oracle's emulation of that arithmetic on the same rows.  The
batched workload (64 problems, complex64 in and out, mixed FP32): 1e-6 plus
the complex64 rounding of y (1e-7) on the stored rows of four problems.
"""
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_plan, rel, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_cache = {}


def run(name, prec):
    import torch
    key = (name, prec)
    if key not in _cache:
        P = W.config(name)
        with gpu_plan(P, prec) as plan:
            y = plan.matvec(to_dev(P.v))
            torch.cuda.synchronize()
            _cache[key] = (y.cpu().numpy(), plan.stats())
        del y
        torch.cuda.empty_cache()
    return _cache[key]


def golden(name, key="y"):
    g = np.load(os.path.join(GOLDEN, f"{name}_rows.npz"))
    return g["rows"], g[key]


@pytest.mark.parametrize("name", ["uniform100k", "uniform1m"])
def test_fp64_sampled_rows(name):
    rows, yo = golden(name)
    y, st = run(name, "fp64")
    assert rel(y[rows], yo) <= 1e-12
    assert np.all(np.isfinite(y))


@pytest.mark.parametrize("name", ["uniform100k", "uniform1m"])
def test_fp32_sampled_rows_and_full_vector(name):
    rows, yo = golden(name)
    y32, st = run(name, "fp32")
    assert rel(y32[rows], yo) <= 1e-6
    y64, _ = run(name, "fp64")
    assert rel(y32, y64) <= 1e-6
    _cache.pop((name, "fp64"), None)


@pytest.mark.parametrize("name", ["uniform100k", "uniform1m"])
def test_bf16x3_sampled_rows(name):
    rows, yo = golden(name)
    _, ye = golden(name, "y_bf16x3")
    y, st = run(name, "bf16x3")
    _cache.pop((name, "bf16x3"), None)
    assert np.all(np.isfinite(y))
    assert rel(y[rows], yo) <= 3 * rel(ye, yo)


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
                    assert rel(yy, g[f"y{i}"]) <= 1e-6 + 1e-7, i
                checked += 1
            assert checked == 4
            for y in ys:
                assert torch.isfinite(torch.view_as_real(y)).all()
    finally:
        for p in plans:
            p.close()
