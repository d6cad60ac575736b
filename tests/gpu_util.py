"""Helpers shared by the GPU tests: run the HIP library on a seeded problem."""
import numpy as np


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device())


def gpu_plan(P, precision="fp64", l_hf=None):
    import paper_2004_14229_amd as F
    pt = to_dev(P.points_T)
    ps = pt if P.same_points else to_dev(P.points_S)
    return F.Plan(pt, ps, P.kappa, P.box, P.levels, P.m, precision=precision, l_hf=l_hf)


def gpu_matvec(P, precision="fp64", plan=None):
    import torch
    plan = plan or gpu_plan(P, precision)
    y = plan.matvec(to_dev(P.v))
    torch.cuda.synchronize()
    return y.cpu().numpy(), plan


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb else 1.0)
