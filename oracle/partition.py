"""Directional admissibility and the block tree (Sect. 2.2-2.3).  Oracle.

Def. of directional admissibility: boxes ``t`` and ``s`` are admissible when

* (A1)  ``max(diam t, diam s) <= eta2 * dist(t, s)`` and
* (A3)  ``kappa * max(diam t, diam s)^2 <= eta2 * dist(t, s)``;

(A2) concerns the direction and is met by construction of the dir maps.
``diam`` is the box diagonal and ``dist`` the Euclidean distance between the
two closed boxes.  For two boxes of one level with integer offset ``o``
(in box units) the gap along axis ``d`` is ``max(|o_d|-1, 0) * h_d``.

Reading taken here: both criteria are compared in squared form in FP64,
``D2 = sum h_d^2``, ``S2 = sum (g_d h_d)^2``, (A1) ``D2 <= eta2^2 S2`` and
(A3) ``kappa^2 D2^2 <= eta2^2 S2``; equality counts as admissible, as printed.
``eta2 = 5`` (the value of Sect. 4).

Alg. 2 builds the block tree from the pair of roots: a pair with a leaf on
either side is a leaf block; otherwise a pair violating (A1) or (A3) is split
into all pairs of children; a pair satisfying both is an admissible leaf.
With adaptive trees (Alg. 1's n_max rule) inadmissible leaf blocks occur on
every level, between a leaf and a box of any size.
The recursion is carried out level by level over arrays of pairs; an optional
target filter keeps only pairs whose target box is listed (exact for the rows
below those boxes, used by the row-sampled oracle).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .tree import BoxTree

ETA2 = 5.0


def admissible(kappa: float, h: np.ndarray, o: np.ndarray,
               eta2: float = ETA2) -> np.ndarray:
    """(A1) and (A3) for same-level boxes with integer offsets ``o``."""
    o = np.asarray(o, dtype=np.int64)
    h = np.asarray(h, dtype=np.float64)
    g = np.maximum(np.abs(o) - 1, 0).astype(np.float64)
    d2 = h[0] * h[0] + h[1] * h[1] + h[2] * h[2]
    s2 = (g[..., 0] * h[0]) ** 2 + (g[..., 1] * h[1]) ** 2 + \
        (g[..., 2] * h[2]) ** 2
    e2 = eta2 * eta2
    a1 = d2 <= e2 * s2
    a3 = (kappa * kappa) * (d2 * d2) <= e2 * s2
    return a1 & a3


@dataclass
class BlockTree:
    levels: int
    adm_t: list  # per level: target box indices of admissible leaves
    adm_s: list  # per level: source box indices of admissible leaves
    near_t: list  # per level: target box of inadmissible leaves
    near_s: list  # per level: source box of inadmissible leaves
    # (uniform trees: only on the last level)

    def n_admissible(self) -> int:
        return int(sum(a.shape[0] for a in self.adm_t))


def block_tree(TT: BoxTree, TS: BoxTree, kappa: float, eta2: float = ETA2,
               target_filter=None) -> BlockTree:
    """Alg. 2 on two depth-``levels`` trees over the same root box.

    ``target_filter``: optional list (per level) of boolean masks over the
    target boxes; pairs whose target is masked out are dropped.
    """
    p = TT.levels
    assert TS.levels == p
    adm_t, adm_s, near_t, near_s = [], [], [], []
    if TT.n == 0 or TS.n == 0:
        e = np.zeros(0, dtype=np.int64)
        return BlockTree(p, [e] * (p + 1), [e] * (p + 1), [e] * (p + 1),
                         [e] * (p + 1))
    t = np.zeros(1, dtype=np.int64)
    s = np.zeros(1, dtype=np.int64)
    h_root = TT.root_hi - TT.root_lo
    for level in range(p + 1):
        if target_filter is not None:
            keep = target_filter[level][t]
            t, s = t[keep], s[keep]
        o = TT.coords[level][t] - TS.coords[level][s]
        ok = admissible(kappa, h_root * 2.0 ** (-level), o, eta2)
        adm_t.append(t[ok])
        adm_s.append(s[ok])
        # a pair with a leaf on either side is a leaf block (inadmissible
        # ones form the near field); other inadmissible pairs are refined
        leaf = TT.is_leaf(level)[t] | TS.is_leaf(level)[s]
        near = ~ok & leaf
        near_t.append(t[near])
        near_s.append(s[near])
        if level == p:  # every box of the last level is a leaf
            break
        refine = ~ok & ~leaf
        rt, rs = t[refine], s[refine]  # refine: all pairs of children
        ct = TT.child_count[level][rt]
        cs = TS.child_count[level][rs]
        npairs = ct * cs
        rep_t = np.repeat(rt, npairs)
        rep_s = np.repeat(rs, npairs)
        first = np.cumsum(npairs) - npairs
        local = np.arange(rep_t.shape[0]) - np.repeat(first, npairs)
        cs_rep = np.repeat(cs, npairs)
        t = TT.child_start[level][rep_t] + local // cs_rep
        s = TS.child_start[level][rep_s] + local % cs_rep
    return BlockTree(p, adm_t, adm_s, near_t, near_s)
