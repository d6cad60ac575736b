"""The C-ABI library loads on a host without a GPU, exports every function
declared in include/fdm.h, and rejects invalid arguments before any device
work (no GPU needed for these paths)."""
import ctypes

import pytest

import paper_2004_14229_amd as F


def test_library_exports_every_declared_symbol():
    names = F.header_functions()
    assert len(names) >= 10
    L = F.lib()
    for n in names:
        assert hasattr(L, n), n
    assert L.fdm_version().startswith(b"fdm-gfx950")


def _build(**kw):
    args = dict(n_T=0, n_S=0, kappa=1.0, box=(0, 0, 0, 1, 1, 1), levels=3, m=4, prec=0, l_hf=-2)
    args.update(kw)
    L = F.lib()
    h = ctypes.c_void_p()
    box = (ctypes.c_double * 6)(*args["box"])
    st = L.fdm_build_tree_ex(None, args["n_T"], None, args["n_S"], args["kappa"], box,
                             args["levels"], args["m"], args["prec"], args["l_hf"], None,
                             ctypes.byref(h))
    return st, h, L.fdm_last_error().decode()


@pytest.mark.parametrize("kw,status", [
    (dict(levels=-1), -1), (dict(levels=10), -1), (dict(m=0), -1), (dict(m=9), -1),
    (dict(kappa=-1.0), -1), (dict(kappa=float("nan")), -1), (dict(prec=7), -1),
    (dict(n_T=-5), -1), (dict(l_hf=5, levels=3), -1),
    (dict(box=(0, 0, 0, 0, 1, 1)), -1), (dict(box=(0, 0, 0, 1, float("inf"), 1)), -1),
    (dict(prec=4), -1), (dict(prec=-1), -1),
    (dict(n_T=2 ** 30), -3), (dict(n_S=2 ** 30), -3), (dict(n_S=-1), -1),
])
def test_invalid_arguments_are_rejected(kw, status):
    st, h, msg = _build(**kw)
    assert st == status and h.value is None and msg


def test_null_handles():
    L = F.lib()
    assert L.fdm_plan_destroy(None) == 0
    assert L.fdm_plan_matvec(None, None, None, None) == -1
    st = F.fdm.Stats()
    assert L.fdm_plan_stats(None, ctypes.byref(st)) == -1
    size = ctypes.c_int64()
    assert L.fdm_plan_export(None, b"perm_T", None, 0, ctypes.byref(size)) == -1


def _build_opts(nb=64, budget=0, prec=0, persistent=1, compact=1, full_bank=0, aca_eps=0.0,
                aca_rank=0, aca_chunk=0, m=4, n_max=0):
    L = F.lib()
    h = ctypes.c_void_p()
    box = (ctypes.c_double * 6)(0, 0, 0, 1, 1, 1)
    opts = F.fdm.Options(prec, -2, budget, F.fdm.Tune(nb, persistent, 1, 0, compact), full_bank,
                         aca_rank, aca_eps, aca_chunk, n_max)
    st = L.fdm_build_tree_opts(None, 0, None, 0, 1.0, box, 3, m, ctypes.byref(opts), None,
                               ctypes.byref(h))
    return st, h, L.fdm_last_error().decode()


@pytest.mark.parametrize("kw", [dict(nb=48), dict(nb=0, budget=-1), dict(budget=1),
                                dict(persistent=2), dict(prec=5), dict(compact=3),
                                dict(compact=-1), dict(full_bank=2), dict(full_bank=-1),
                                dict(prec=1, aca_eps=-1.0), dict(prec=1, aca_eps=float("inf")),
                                dict(prec=1, aca_eps=1e-6, aca_rank=48),
                                dict(prec=1, aca_eps=1e-6, budget=1 << 30),
                                dict(prec=1, aca_eps=1e-6, aca_chunk=-1), dict(n_max=-1)])
def test_invalid_options_are_rejected(kw):
    st, h, msg = _build_opts(**kw)
    assert st == -1 and h.value is None and msg


@pytest.mark.parametrize("prec", [0, 2, 3])
def test_low_rank_couplings_need_fp32(prec):
    st, h, msg = _build_opts(prec=prec, aca_eps=1e-6)
    assert st == -3 and h.value is None and "FP32" in msg


@pytest.mark.parametrize("m", [7, 8])
def test_low_rank_couplings_need_m_at_most_6(m):
    st, h, msg = _build_opts(prec=1, aca_eps=1e-6, m=m)
    assert st == -3 and h.value is None and "m <= 6" in msg


def test_null_handles_are_rejected():
    L = F.lib()
    t = F.fdm.Tune(64, 1, 1, 0, 1)
    assert L.fdm_plan_set_tune(None, ctypes.byref(t), None) == -1
    assert L.fdm_plan_get_tune(None, ctypes.byref(t)) == -1
    out = ctypes.c_void_p()
    assert L.fdm_batch_create(None, 0, 0, None, ctypes.byref(out)) == -1
    assert out.value is None
    assert L.fdm_batch_matvec(None, None, None, 0, None) == -1
    assert L.fdm_batch_destroy(None) == 0
    assert L.fdm_plan_autotune(None, None, None, 0, 1, None, None, None) == -1
