"""Write the stored expected values of the full-size parity tests.

Calls only the oracle (and the seeded input generators): for each named
workload, Alg. 4 of the oracle (FP64) evaluated at a sample of target rows,
saved as ``<workload>_rows.npz`` with ``rows`` (user indices), ``y``
(complex128) and ``y_bf16x3`` / ``y_bf16x6``: the same rows with the
coupling products emulated in the BF16 split precisions (``oracle.emulate``),
which fix the expected error of those precisions.  The sample is a seeded
random draw plus, for the uniform workloads, the targets nearest to the
corners, the face centres and the centre of the root box (leaves at the
domain boundary, where blocks have the fewest partners, and in the middle,
where they have the most).  Run from the repository root:

    python tests/golden/make_golden.py uniform100k uniform1m paper_k6 uniform4m
    python tests/golden/make_golden.py degree7 degree8
    python tests/golden/make_golden.py batch

``degree7`` / ``degree8``: small problems at m = 7 and 8, every row.

``batch``: the batched workload (64 problems of ``workloads.batch_problems``),
oracle rows of four of its problems (two uniform, two clustered), saved as
``batch_rows.npz`` with ``rows<i>`` and ``y<i>`` for problem i.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

SAMPLES = {"uniform100k": 64, "uniform1m": 256, "uniform4m": 32, "paper_k6": 256}
# small workloads stored whole (every target row)
WHOLE = ("degree7", "degree8")
MODES = ("fp64", "bf16x3", "bf16x6")
BATCH_GOLDEN = (2, 4, 35, 46)  # problem indices in workloads.batch_problems()
BATCH_ROWS = 16


def landmark_rows(P) -> np.ndarray:
    """Targets nearest to the 8 corners, the 6 face centres and the centre
    of the root box."""
    lo, hi = np.asarray(P.box[:3]), np.asarray(P.box[3:])
    marks = [lo + (hi - lo) * np.array(f) for f in
             [(i, j, k) for i in (0, 1) for j in (0, 1) for k in (0, 1)] +
             [(0, .5, .5), (1, .5, .5), (.5, 0, .5), (.5, 1, .5), (.5, .5, 0), (.5, .5, 1),
              (.5, .5, .5)]]
    return np.array([int(np.argmin(np.sum((P.points_T - q) ** 2, axis=1))) for q in marks])


def sample(name: str, R: int) -> np.ndarray:
    P = W.config(name)
    if name in WHOLE:
        return np.arange(P.points_T.shape[0])
    rows = np.random.default_rng(12345).choice(P.points_T.shape[0], R, replace=False)
    if name != "uniform100k":  # (its stored sample predates the landmarks)
        rows = np.concatenate([rows, landmark_rows(P)])
    return np.unique(rows)


def batch() -> None:
    probs = W.batch_problems()
    out = {}
    for i in BATCH_GOLDEN:
        P = probs[i]
        rows = np.sort(np.random.default_rng(1000 + i).choice(P.points_T.shape[0], BATCH_ROWS,
                                                              replace=False))
        t = time.time()
        plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m, rows=rows)
        out[f"rows{i}"] = rows
        out[f"y{i}"] = oracle.matvec(plan, P.v)
        print(f"batch problem {i}: N={P.points_T.shape[0]} {len(rows)} rows in "
              f"{time.time() - t:.1f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_rows.npz")
    np.savez(path, **out)
    print(f"-> {path}")


def main(names):
    if "batch" in names:
        batch()
        names = [n for n in names if n != "batch"]
    for name in names:
        P = W.config(name)
        rows = sample(name, SAMPLES.get(name, 0))
        t = time.time()
        plan = oracle.build(P.points_T, P.points_S, P.kappa, P.box, P.levels, P.m,
                            rows=rows)
        ys = oracle.matvec(plan, P.v, m2l=MODES)
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_rows.npz")
        np.savez(out, rows=rows, y=ys[0], **{f"y_{mode}": y for mode, y in zip(MODES[1:], ys[1:])})
        print(f"{name}: {len(rows)} rows in {time.time() - t:.1f} s -> {out}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["uniform100k", "uniform1m"])
