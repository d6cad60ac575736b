"""Uniform box cluster trees (Sect. 2.1, Alg. 1).  Oracle: test infrastructure.

Alg. 1 refines a half-open box ``(a_1,b_1] x (a_2,b_2] x (a_3,b_3]`` by
splitting it at its centre ``c_d = (a_d + b_d)/2`` into 8 children, keeping
only children that contain a point, and recursing.

Readings taken here (the paper leaves them open):

* Stop rule.  Alg. 1 refines a box while it holds more than ``n_max``
  points.  Here the depth is also capped at ``levels`` (a box at that level is
  a leaf whatever its count; Alg. 1 alone never stops on coincident points).
  ``n_max=None`` refines every non-empty box down to ``levels``, so all
  leaves sit on that level: the uniform octrees of fixed depth that the
  paper's own tests use (Sect. 4).  With ``n_max`` given, leaves sit on
  several levels (an adaptive tree).
* A point ``x`` lies in the upper child along axis ``d`` iff ``x_d > c_d``
  (the boxes are half-open at the lower end), with ``c_d`` computed as
  ``0.5*(lo_d + hi_d)`` from the parent's bounds, level by level.
* Child numbering: octant ``4*[x>c_1] + 2*[y>c_2] + [z>c_3]`` (so ``T_1`` is
  the lower corner and ``T_8`` the upper, as in Alg. 1).  The Morton key of a
  box is its octant path read as base-8 digits, root first.
* Boxes of a level are ordered by Morton key; points are ordered by the key of
  their leaf, ties broken by the input index.

The tree is built level by level (all boxes of one level at once) rather than
depth first; the set of boxes and their index sets are the same.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class BoxTree:
    levels: int
    root_lo: np.ndarray  # (3,)
    root_hi: np.ndarray  # (3,)
    perm: np.ndarray  # (n,) int64: tree slot -> input index
    points: np.ndarray  # (n, 3) points in tree order
    keys: list  # per level: (nb,) int64 Morton keys, ascending
    start: list  # per level: (nb,) int64 first tree slot of the box
    count: list  # per level: (nb,) int64 number of points (#t-hat)
    coords: list  # per level: (nb, 3) int64 integer box position
    lo: list  # per level: (nb, 3) lower box bounds
    hi: list  # per level: (nb, 3) upper box bounds
    parent: list  # per level: (nb,) index of the parent box (-1 at level 0)
    child_start: list  # per level: (nb,) index of the first child box
    child_count: list  # per level: (nb,) number of children

    @property
    def n(self) -> int:
        return self.perm.shape[0]

    def side(self, level: int) -> np.ndarray:
        """Side lengths of every box at ``level`` (boxes are translates)."""
        return (self.root_hi - self.root_lo) * 2.0 ** (-level)

    def centres(self, level: int) -> np.ndarray:
        return 0.5 * (self.lo[level] + self.hi[level])

    def is_leaf(self, level: int) -> np.ndarray:
        """Leaves of ``level``: boxes without children."""
        return self.child_count[level] == 0

    def box_of_slots(self, level: int, slots: np.ndarray) -> np.ndarray:
        """Box of ``level`` holding each tree slot, -1 where the slot lies
        below a leaf of a coarser level."""
        slots = np.asarray(slots, dtype=np.int64)
        b = np.searchsorted(self.start[level], slots, side="right") - 1
        ok = b >= 0
        bb = np.where(ok, b, 0)
        ok &= slots < self.start[level][bb] + self.count[level][bb]
        return np.where(ok, b, -1)


def _deinterleave(keys: np.ndarray, level: int) -> np.ndarray:
    """Integer (ix, iy, iz) box position from a level-``level`` Morton key."""
    c = np.zeros((keys.shape[0], 3), dtype=np.int64)
    for i in range(level):  # digit i (root first) is octant at level i+1
        shift = 3 * (level - 1 - i)
        octant = (keys >> shift) & 7
        w = 1 << (level - 1 - i)
        c[:, 0] += ((octant >> 2) & 1) * w
        c[:, 1] += ((octant >> 1) & 1) * w
        c[:, 2] += (octant & 1) * w
    return c


def check_inside(points: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> None:
    pts = np.asarray(points, dtype=np.float64)
    if pts.size and (np.any(pts <= lo) or np.any(pts > hi) or
                     not np.all(np.isfinite(pts))):
        raise ValueError("point outside the half-open root box (a, b]")


def build_box_tree(points, box, levels: int, n_max: int | None = None) -> BoxTree:
    """Alg. 1: a non-empty box is refined while it holds more than ``n_max``
    points and lies above level ``levels`` (``n_max=None``: every non-empty
    box above ``levels``)."""
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 3))
    root_lo = np.asarray(box[:3], dtype=np.float64)
    root_hi = np.asarray(box[3:], dtype=np.float64)
    if levels < 0:
        raise ValueError("levels must be >= 0")
    check_inside(pts, root_lo, root_hi)
    n = pts.shape[0]

    # Per point: walk down the levels, comparing with the current box centre.
    lo = np.broadcast_to(root_lo, (n, 3)).copy()
    hi = np.broadcast_to(root_hi, (n, 3)).copy()
    leaf_key = np.zeros(n, dtype=np.int64)
    for _ in range(levels):
        c = 0.5 * (lo + hi)
        upper = pts > c
        lo = np.where(upper, c, lo)
        hi = np.where(upper, hi, c)
        octant = 4 * upper[:, 0] + 2 * upper[:, 1] + upper[:, 2]
        leaf_key = leaf_key * 8 + octant.astype(np.int64)

    perm = np.lexsort((np.arange(n, dtype=np.int64), leaf_key))
    sorted_key = leaf_key[perm]

    keys, start, count, coords = [], [], [], []
    for level in range(levels + 1):
        k = sorted_key >> (3 * (levels - level))
        if n:
            first = np.concatenate(([True], k[1:] != k[:-1]))
        else:
            first = np.zeros(0, dtype=bool)
        st = np.flatnonzero(first).astype(np.int64)
        kk = k[st]
        cnt = np.diff(np.concatenate((st, [n]))).astype(np.int64)
        if n_max is not None and level > 0:
            # a box exists if its parent exists and holds more than n_max
            # points (the boxes of the previous level are those that exist)
            pk = kk >> 3
            npar = keys[level - 1].shape[0]
            exists = np.zeros(kk.shape[0], dtype=bool)
            if npar:
                pi = np.minimum(np.searchsorted(keys[level - 1], pk), npar - 1)
                exists = (keys[level - 1][pi] == pk) & (count[level - 1][pi] > n_max)
            st, kk, cnt = st[exists], kk[exists], cnt[exists]
        keys.append(kk)
        start.append(st)
        count.append(cnt)
        coords.append(_deinterleave(kk, level))

    # Box bounds from the same centre recursion as the point classification.
    blo = [root_lo[None, :].copy() if n else np.zeros((0, 3))]
    bhi = [root_hi[None, :].copy() if n else np.zeros((0, 3))]
    parent = [np.full(keys[0].shape[0], -1, dtype=np.int64)]
    child_start, child_count = [], []
    for level in range(1, levels + 1):
        pkeys = keys[level] >> 3
        par = np.searchsorted(keys[level - 1], pkeys)
        parent.append(par.astype(np.int64))
        octant = keys[level] & 7
        plo = blo[level - 1][par]
        phi = bhi[level - 1][par]
        c = 0.5 * (plo + phi)
        upper = np.stack([(octant >> 2) & 1, (octant >> 1) & 1, octant & 1],
                         axis=1).astype(bool)
        blo.append(np.where(upper, c, plo))
        bhi.append(np.where(upper, phi, c))
        nparent = keys[level - 1].shape[0]
        cs = np.searchsorted(par, np.arange(nparent))
        cc = np.bincount(par, minlength=nparent)
        child_start.append(cs.astype(np.int64))
        child_count.append(cc.astype(np.int64))
    nleaf = keys[levels].shape[0]
    child_start.append(np.zeros(nleaf, dtype=np.int64))
    child_count.append(np.zeros(nleaf, dtype=np.int64))

    return BoxTree(levels, root_lo, root_hi, perm.astype(np.int64), pts[perm],
                   keys, start, count, coords, blo, bhi, parent,
                   child_start, child_count)
