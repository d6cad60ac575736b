"""Host-side accounting of bench.py (no GPU): the compulsory HBM bytes of
the transfer phases, counted by hand for a small two-level tree."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_hbm_phase_bytes_by_hand(bench):
    # levels 0..2, couplings from level 1; K = 27 -> Kp = 32
    shape = {"nbS": [1, 4, 10], "nbT": [1, 3, 7], "nd": [1, 2, 1], "levels": 2, "l_min": 1}
    nT, nS, K = 50, 40, 27
    ms = {"s2m": 1.0, "m2m": 2.0, "l2l": 4.0, "l2t": 0.5, "near": 0.001}
    r = bench.hbm_phases(shape, ms, K, nT, nS, mixed=True)
    vec, mom_w = 32 * 16, 32 * 16 + 32 * 8
    assert r["s2m"]["bytes"] == 16 * nS * 2 + 40 * nS + 10 * 1 * mom_w
    assert r["m2m"]["bytes"] == 10 * 1 * vec + 4 * 2 * mom_w  # level 2 -> 1 only
    assert r["l2l"]["bytes"] == 3 * 2 * vec + 7 * 1 * 2 * vec
    assert r["l2t"]["bytes"] == 7 * vec + 24 * nT + 32 * nT
    assert r["near"]["bytes"] == 24 * nT + 40 * nS + 16 * nT
    assert r["m2m"]["GB/s"] == pytest.approx(r["m2m"]["bytes"] / 2e-3 / 1e9)
    assert r["near"]["GB/s"] is None  # a phase below 10 us gets no rate
    plain = bench.hbm_phases(shape, ms, K, nT, nS, mixed=False)
    assert plain["m2m"]["bytes"] == 10 * vec + 4 * 2 * vec



def test_traffic_only_for_the_measured_kernel_source(bench, tmp_path, monkeypatch):
    """The counter record gives `traffic` only while its SHA-256 matches the
    kernel's current sources; a stale or missing record gives null."""
    csrc = tmp_path / "paper_2004_14229_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (csrc / "m2l_device.hpp").write_text("// shared\n")
    (csrc / "m2l_f32.hip").write_text("// fp32\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_for("k_m2l_f32", "w", 1.0) is None  # no record
    rec = tmp_path / "profiles" / "k_m2l_f32_w_counters.json"
    sha = bench.kernel_source_sha("k_m2l_f32")
    rec.write_text('{"source_sha256": "%s", "hbm_bytes_per_launch": 123.5}' % sha)
    assert bench.traffic_for("k_m2l_f32", "w", 1.0) == 123.5
    (csrc / "m2l_device.hpp").write_text("// shared, edited\n")
    assert bench.traffic_for("k_m2l_f32", "w", 1.0) is None


def _oracle_counts(P):
    """Work counts of a whole problem from the oracle's own plan, in the
    form bench.py takes them from the GPU plan."""
    import oracle
    plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m)
    st = oracle.structure(plan)
    nc = [int(st[f"nc{l}"][0]) for l in range(P.levels + 1)]
    l_min = min([l for l in range(P.levels + 1) if nc[l]] or [P.levels + 1])
    shape = {"nbS": [int(plan.TS.keys[l].shape[0]) for l in range(P.levels + 1)],
             "nbT": [int(plan.TT.keys[l].shape[0]) for l in range(P.levels + 1)],
             "nd": [int(plan.dirs.vectors(l).shape[0]) if l >= l_min else 1
                    for l in range(P.levels + 1)],
             "levels": P.levels, "l_min": l_min}
    stats = {"n_couplings": sum(nc),
             "n_stored_couplings": sum(int(st[f"off{l}"].shape[0]) for l in range(P.levels + 1)),
             "near_entries": int(st["near_entries"][0])}
    return shape, stats


def test_cpu_baseline_whole_problem_is_not_scaled(bench):
    """With the whole box as the sample, every phase's work count equals the
    workload's, so each extrapolated phase time is the measured one."""
    import workloads as W
    P = W.config("uniform2k")
    shape, stats = _oracle_counts(P)
    r = bench.cpu_baseline(P, stats, shape, sub_div=1)
    assert r["kind"] == "oracle" and r["unit"] == "matvecs/s" and r["cores"] >= 1
    for k, ph in r["phases"].items():
        assert ph["extrapolated_s"] == pytest.approx(ph["sample_s"], rel=1e-9, abs=1e-12), k
    assert r["extrapolated_s_per_matvec"] == pytest.approx(
        sum(ph["sample_s"] for ph in r["phases"].values()))


def test_cpu_baseline_sub_cube_sample(bench):
    """The sample is the sub-cube (0, 1/2]^3 with one level less: its work
    counts are a fraction of the workload's and scale up each phase."""
    import workloads as W
    P = W.config("uniform2k")
    shape, stats = _oracle_counts(P)
    r = bench.cpu_baseline(P, stats, shape, sub_div=2)
    assert r["value"] > 0 and "sub-cube (0,0.5]^3" in r["sample"]
    for k in ("s2m", "l2t", "near", "m2m", "l2l"):
        ph = r["phases"][k]
        assert 0 < ph["sample_units"] < ph["full_units"], k
    assert r["phases"]["m2l"]["sample_blocks"] < stats["n_couplings"]
