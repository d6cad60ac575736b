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
    (dict(box=(0, 0, 0, 1, 1, 2)), -3), (dict(box=(0, 0, 0, 0, 1, 1)), -1),
    (dict(m=7), -3), (dict(prec=3), -1), (dict(prec=-1), -1),
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
