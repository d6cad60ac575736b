"""The Python binding checks tensors before any pointer reaches the library
(which sees no sizes): host tensors, wrong dtypes and wrong lengths raise
TypeError on every entry that takes vectors, with no device work."""
import numpy as np
import pytest
import torch

import paper_2004_14229_amd as F


def _plan(n_T=5, n_S=4):
    p = object.__new__(F.Plan)  # no device plan: the checks come first
    p._h, p.n_T, p.n_S, p.precision = None, n_T, n_S, "fp64"
    return p


@pytest.mark.parametrize("v", [
    np.zeros(4, np.complex128),
    torch.zeros(4, dtype=torch.complex128),           # host tensor
    torch.zeros(4, dtype=torch.float64),
])
def test_plan_vectors_rejected(v):
    p = _plan()
    with pytest.raises(TypeError):
        p.matvec(v)
    with pytest.raises(TypeError):
        p.autotune(v)


def test_batch_vectors_rejected():
    b = object.__new__(F.Batch)
    b._h, b.plans = None, [_plan(), _plan(3, 2)]
    with pytest.raises(ValueError):
        b.matvec([torch.zeros(4, dtype=torch.complex128)])
    with pytest.raises(TypeError):
        b.matvec([torch.zeros(4, dtype=torch.complex128), torch.zeros(2, dtype=torch.complex128)])
    with pytest.raises(TypeError):
        b.autotune([torch.zeros(4, dtype=torch.int64), torch.zeros(2, dtype=torch.int64)])


def test_dense_and_plan_points_rejected():
    pts = torch.zeros(3, 3, dtype=torch.float64)
    with pytest.raises(TypeError):
        F.dense_matvec(pts, pts, 1.0, torch.zeros(3, dtype=torch.complex128))
    with pytest.raises(TypeError):
        F.Plan(pts, pts, 1.0, (0, 0, 0, 1, 1, 1), 2, 2)
