"""Pins of the oracle's reduced-precision emulation (``oracle.emulate``),
which fixes the expected error of the mixed-precision coupling products:
BF16 rounding against torch's float32 -> bfloat16 conversion and hand-made
ties, the split error bounds, and the products on inputs whose parts and
sums are exact in FP32, where each mode's result is known in closed form
(the BF16 split with three products drops exactly the lo*lo term)."""
import numpy as np
import pytest
import torch

from oracle import emulate as E


def test_round_bf16_matches_library_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-20, 20, 20000),
        # exact ties: low 16 bits 0x8000, both parities of the kept bit
        (rng.integers(0x3F000000, 0x40800000, 4000, dtype=np.uint32) & 0xFFFF0000 | 0x8000).view(np.float32),
    ]).astype(np.float32)
    x = np.concatenate([x, -x])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(E.round_bf16(x), want)


@pytest.mark.parametrize("x,want", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                      # tie, kept bit even: down
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),      # tie, kept bit odd: up
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # above the tie: up
    (-(1.0 + 3 * 2.0 ** -8), -(1.0 + 2.0 ** -6)),
    (3.0, 3.0), (0.0, 0.0),
])
def test_round_bf16_ties_to_even(x, want):
    assert float(E.round_bf16(np.float32(x))) == want


def test_split_error_bounds():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(50000) * 10.0 ** rng.uniform(-8, 8, 50000)
    x32 = x.astype(np.float32)
    hi, lo = E.split_bf16(x32)
    assert np.array_equal(E.round_bf16(hi), hi) and np.array_equal(E.round_bf16(lo), lo)
    r2 = np.abs(x32.astype(np.float64) - hi - lo) / np.abs(x32)
    assert r2.max() <= 2.0 ** -17          # two roundings of 2^-9 each
    assert r2.max() > 2.0 ** -22           # and not exact: lo*lo terms matter
    h, m, l = E.split3_bf16(x)
    for part in (h, m, l):
        assert np.array_equal(E.round_bf16(part), part)
    r3 = np.abs(x - h.astype(np.float64) - m - l) / np.abs(x)
    assert r3.max() <= 2.0 ** -25


def _exact_parts(rng, shape):
    """Values hi + lo with hi an integer in [8, 16) (sign random) and lo a
    multiple of 2^-12 below 2^-9: both BF16, and hi = round_bf16(hi + lo)."""
    hi = rng.integers(8, 16, shape) * rng.choice([-1.0, 1.0], shape)
    lo = rng.integers(-7, 8, shape) * 2.0 ** -12
    return hi, lo


def test_products_closed_form_on_exact_parts():
    """K = 4 terms.  The split parts are the constructed hi and lo, and every
    partial product of parts and their sums in the BF16 split modes are
    exact in FP32 (at most 23 significant bits), so bf16x3 gives the exact
    product minus the lo*lo cross terms, bit for bit; bf16x6 and fp32 give
    the exact product to FP32 rounding (here the lo*lo terms are below the
    last bit of the FP32 sums, so bf16x6 may lose them too)."""
    rng = np.random.default_rng(2)
    n, k, q = 5, 4, 3  # M (n, k), A (q, k): product M @ A.T is (n, q)
    Arh, Arl = _exact_parts(rng, (q, k))
    Aih, Ail = _exact_parts(rng, (q, k))
    Mrh, Mrl = _exact_parts(rng, (n, k))
    Mih, Mil = _exact_parts(rng, (n, k))
    A = (Arh + Arl) + 1j * (Aih + Ail)
    M = (Mrh + Mrl) + 1j * (Mih + Mil)
    exact = M @ A.T
    for p, ref in ((Arh, Arh), (Arl, Arl)):
        assert np.array_equal(E.round_bf16(p.astype(np.float32)), ref)
    hi_r, lo_r = E.split_bf16((Arh + Arl).astype(np.float32))
    assert np.array_equal(hi_r, Arh) and np.array_equal(lo_r, Arl)

    assert np.array_equal(E.product(A, M, "fp64"), exact)
    # the entries (16 bits) are exact in FP32, their products (up to 32 bits)
    # are not: FP32 gives the product to FP32 rounding
    got32 = E.product(A, M, "fp32").astype(np.complex128)
    assert np.abs(got32 - exact).max() <= 4 * k * 2.0 ** -24 * np.abs(exact).max()
    lolo = (Mrl @ Arl.T - Mil @ Ail.T) + 1j * (Mrl @ Ail.T + Mil @ Arl.T)
    assert np.abs(lolo).max() > 0
    got3 = E.product(A, M, "bf16x3").astype(np.complex128)
    assert np.array_equal(got3, exact - lolo)
    got6 = E.product(A, M, "bf16x6").astype(np.complex128)
    assert np.abs(got6 - exact).max() <= 4 * k * 2.0 ** -24 * np.abs(exact).max()


def test_product_error_on_random_operands():
    """Relative error of each mode against FP64 on random complex operands
    (K = 343, the coupling size at m = 6) lies in the band its arithmetic
    predicts: FP32 rounding of products and sums (~2^-22); the dropped
    lo*lo term of the three-product split (each 2^-18 of a product, ~2^-18);
    the six-product split keeps it, with exact BF16 part products and only
    the FP32 sums rounding, so it ends below FP32."""
    rng = np.random.default_rng(3)
    K = 343
    A = rng.standard_normal((40, K)) + 1j * rng.standard_normal((40, K))
    M = rng.standard_normal((30, K)) + 1j * rng.standard_normal((30, K))
    ref = M @ A.T
    err = {mode: np.linalg.norm(E.product(A, M, mode).astype(np.complex128) - ref)
           / np.linalg.norm(ref) for mode in ("fp32", "bf16x3", "bf16x6")}
    assert 2.0 ** -23 <= err["fp32"] <= 2.0 ** -20.5, err
    assert 2.0 ** -19 <= err["bf16x3"] <= 2.0 ** -16.5, err
    assert 2.0 ** -25 <= err["bf16x6"] <= 2.0 ** -22, err
    assert err["bf16x6"] < err["fp32"] < err["bf16x3"]


def test_accumulation_type():
    assert E.accumulate_dtype("fp32") == np.complex64
    for mode in ("fp64", "fp32acc64", "bf16x3", "bf16x6"):
        assert E.accumulate_dtype(mode) == np.complex128
    with pytest.raises(ValueError):
        E.product(np.ones((2, 2)), np.ones((2, 2)), "fp16")


def test_emulated_matvec_errors_follow_the_arithmetic():
    """Alg. 4 with the coupling step emulated in each mode: FP32 products
    stay near FP32 rounding (and summing the offsets in FP64 is no worse),
    the three-product BF16 split is an order of magnitude above, the
    six-product split back at FP32 level."""
    import oracle
    import workloads as W
    P = W.random_problem(52, 400, 380, 30.0, 3, 4)
    plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m)
    y = oracle.matvec(plan, P.v)
    err = {mode: np.linalg.norm(oracle.matvec(plan, P.v, m2l=mode) - y) / np.linalg.norm(y)
           for mode in ("fp32", "fp32acc64", "bf16x3", "bf16x6")}
    assert 1e-8 <= err["fp32"] <= 1e-6, err
    assert err["fp32acc64"] <= err["fp32"], err
    assert 5e-7 <= err["bf16x3"] <= 1e-5 and err["bf16x3"] >= 5 * err["fp32"], err
    assert err["bf16x6"] <= err["fp32"], err
