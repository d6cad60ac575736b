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


def assert_close(a, b, tol, what=""):
    """Relative l2 error at most tol, and every entry within tol times the
    largest reference entry (a few wrong entries cannot hide in the norm)."""
    a = np.asarray(a)
    b = np.asarray(b)
    err = rel(a, b)
    assert err <= tol, f"{what} rel l2 {err:.3e} > {tol:.3e}"
    scale = np.max(np.abs(b)) if b.size else 0.0
    worst = np.max(np.abs(a - b)) if a.size else 0.0
    assert worst <= tol * (scale if scale else 1.0), \
        f"{what} max |diff| {worst:.3e} > {tol:.3e} * max |ref| {scale:.3e}"
    return err
