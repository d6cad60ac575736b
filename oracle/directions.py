"""Directions (Sect. 2.4, Alg. 3, Def. of dir maps; Sect. 2.6 Def. of active
and inherited directions).  Oracle: test infrastructure.

Alg. 3: ``D^(l) = {0}`` on low-frequency levels ``l > l_hf``; at ``l_hf`` the
six faces of ``[-1,1]^3`` and their centres; each coarser level splits every
face of the finer level into 4 and takes the normalised midpoints, so
``#D^(l) = 6 * 4^(l_hf - l)``.  ``dir_(l)(v)`` is the direction of the face
(lowest index among the closed faces) hit by the ray through ``v``.

Readings taken here:

* ``l_hf``: the largest level ``l <= levels`` with ``kappa * h_l >= 3.2``
  (``h_l`` the box side), else -1.  This is the high-frequency condition of
  Sect. 2.4 with ``eta_1 = 3.2 sqrt(3)``; it gives ``l_hf = k - 4`` in the
  setting of Sect. 4.
* Face order at ``l_hf``: ``{x=-1}, {x=+1}, {y=-1}, {y=+1}, {z=-1}, {z=+1}``.
* The 4 sub-faces of a face are ordered like a quadtree over the face's two
  free axes (lower axis = more significant bit), with each free coordinate
  measured along ``sign(face) * e_b`` (mirrored on the three negative faces).
  This makes ``dir(-v) = -dir(v)``.
* Membership of ``psi_Q(v) = v / max|v_j|`` in a closed face is decided in
  exact integer arithmetic: the argument is an integer offset between box
  centres (cubic boxes), or a face midpoint, which is dyadic.  For a
  non-cubic root box the centre offset is ``o * h`` with the box sides
  ``h``: floating-point sides are dyadic rationals, so ``o * h`` times a
  common power of two is an integer vector, and the same exact test
  applies (Python integers).
* ``l_hf`` for a non-cubic root box uses the longest side.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

TAU_HF = 3.2


def high_frequency_level(kappa: float, side: float, levels: int,
                         tau: float = TAU_HF) -> int:
    l_hf = -1
    for level in range(levels + 1):
        if kappa * (side * 2.0 ** (-level)) >= tau:
            l_hf = level
    return l_hf


@dataclass
class FaceSet:
    """Faces ``E_j^(l)`` of one level as exact dyadic rectangles.

    Coordinates are integers over the common denominator ``den``.
    """
    den: int
    axis: np.ndarray  # (nf,) fixed axis a
    sign: np.ndarray  # (nf,) +1 / -1
    lo: np.ndarray  # (nf, 3) lower bounds (numerators); axis a: sign*den
    hi: np.ndarray  # (nf, 3) upper bounds (numerators)

    def midpoints(self) -> np.ndarray:
        """Face midpoints as integers over denominator ``2*den``."""
        return self.lo + self.hi

    def directions(self) -> np.ndarray:
        mid = self.midpoints().astype(np.float64)
        return mid / np.linalg.norm(mid, axis=1, keepdims=True)


def _top_faces() -> FaceSet:
    axis = np.array([0, 0, 1, 1, 2, 2])
    sign = np.array([-1, 1, -1, 1, -1, 1])
    lo = -np.ones((6, 3), dtype=np.int64)
    hi = np.ones((6, 3), dtype=np.int64)
    for j in range(6):
        lo[j, axis[j]] = hi[j, axis[j]] = sign[j]
    return FaceSet(1, axis, sign, lo, hi)


def _subdivide(F: FaceSet) -> FaceSet:
    """Split each face into 4 (Alg. 3, inner loop), children in face order."""
    den = 2 * F.den
    axis, sign, lo, hi = [], [], [], []
    for j in range(F.axis.shape[0]):
        a, sg = int(F.axis[j]), int(F.sign[j])
        flo, fhi = 2 * F.lo[j], 2 * F.hi[j]
        mid = (flo + fhi) // 2
        free = [b for b in range(3) if b != a]
        for q in range(4):
            bits = ((q >> 1) & 1, q & 1)  # lower free axis is the high bit
            clo, chi = flo.copy(), fhi.copy()
            for b, beta in zip(free, bits):
                # beta = 0 is the half that comes first along sign*e_b
                lower_half = (sg > 0) == (beta == 0)
                if lower_half:
                    chi[b] = mid[b]
                else:
                    clo[b] = mid[b]
            axis.append(a)
            sign.append(sg)
            lo.append(clo)
            hi.append(chi)
    return FaceSet(den, np.array(axis), np.array(sign), np.array(lo),
                   np.array(hi))


class DirectionSets:
    """``D^(l)`` for ``l = 0..levels`` and the maps ``dir_(l)``."""

    def __init__(self, l_hf: int, levels: int):
        self.l_hf = l_hf
        self.levels = levels
        self.faces = {}
        if l_hf >= 0:
            F = _top_faces()
            self.faces[l_hf] = F
            for level in range(l_hf - 1, -1, -1):
                F = _subdivide(F)
                self.faces[level] = F

    def count(self, level: int) -> int:
        """Number of stored directions at ``level`` (1 for ``{0}``)."""
        if level > self.l_hf:
            return 1
        return 6 * 4 ** (self.l_hf - level)

    def vectors(self, level: int) -> np.ndarray:
        if level > self.l_hf:
            return np.zeros((1, 3))
        return self.faces[level].directions()

    def dir_index(self, level: int, v: np.ndarray) -> np.ndarray:
        """Index of ``dir_(level)(v)`` for integer vectors ``v`` (..., 3).

        Returns 0 on low-frequency levels (the single direction ``0``) and -1
        for ``v = 0`` on high-frequency levels.
        """
        v = np.asarray(v)
        if v.dtype != object:
            v = v.astype(np.int64)
        shape = v.shape[:-1]
        v = v.reshape(-1, 3)
        if level > self.l_hf:
            return np.zeros(shape, dtype=np.int64)
        F = self.faces[level]
        M = np.abs(v).max(axis=1)  # psi_Q(v) = v / M
        # psi_Q(v) in face j  <=>  v_a = sign*M  and  lo_b*M <= v_b*den <= hi_b*M
        vv = v[:, None, :]
        MM = M[:, None, None]
        inside = (vv * F.den >= F.lo[None] * MM) & (vv * F.den <= F.hi[None] * MM)
        member = inside.all(axis=2)
        member &= (M[:, None] > 0)
        j = np.where(member.any(axis=1), member.argmax(axis=1), -1)
        return j.reshape(shape)

    def parent_index(self, level: int) -> np.ndarray:
        """``dir_(level+1)(c)`` for every ``c`` in ``D^(level)`` (Sect. 2.5)."""
        if level + 1 > self.l_hf:
            return np.zeros(self.count(level), dtype=np.int64)
        mids = self.faces[level].midpoints()  # dyadic, integer numerators
        return self.dir_index(level + 1, mids)


def exact_offsets(o: np.ndarray, side) -> np.ndarray:
    """Box-centre offsets ``o * h`` (``o`` integer, ``h`` the side lengths at
    any level) as exact integer vectors up to one positive factor; ``o``
    itself for equal sides."""
    side = np.asarray(side, dtype=np.float64).reshape(3)
    if side[0] == side[1] == side[2]:
        return o
    fr = [Fraction(float(x)) for x in side]
    den = math.lcm(*[f.denominator for f in fr])
    S = [int(f * den) for f in fr]
    o = np.asarray(o, dtype=np.int64).reshape(-1, 3)
    out = np.empty(o.shape, dtype=object)
    for d in range(3):
        out[:, d] = [int(a) * S[d] for a in o[:, d]]
    return out


def active_directions(TT, TS, BT, dirs: DirectionSets, side):
    """Def. of active and inherited directions for both trees.

    Returns ``(DT, DhT, DS, DhS)``, each a list over levels of boolean arrays
    ``[n_boxes, #D^(l)]``, and ``cdir`` (per level, the direction index of
    every admissible block).
    """
    p = TT.levels
    DT, DS, cdir = [], [], []
    for level in range(p + 1):
        nd = dirs.count(level)
        dt = np.zeros((TT.keys[level].shape[0], nd), dtype=bool)
        ds = np.zeros((TS.keys[level].shape[0], nd), dtype=bool)
        t, s = BT.adm_t[level], BT.adm_s[level]
        o = TT.coords[level][t] - TS.coords[level][s]  # (m_t - m_s) / h
        c = dirs.dir_index(level, exact_offsets(o, TT.root_hi - TT.root_lo))
        dt[t, c] = True
        ds[s, c] = True
        DT.append(dt)
        DS.append(ds)
        cdir.append(c)

    def inherit(T, D):
        Dh = [np.zeros_like(D[0])]
        for level in range(1, p + 1):
            up = D[level - 1] | Dh[level - 1]  # over parent boxes
            par_dir = dirs.parent_index(level - 1)  # dir_(level)(c)
            nd = dirs.count(level)
            dh = np.zeros((T.keys[level].shape[0], nd), dtype=bool)
            inh = np.zeros((up.shape[0], nd), dtype=bool)
            for cp in range(up.shape[1]):
                inh[:, par_dir[cp]] |= up[:, cp]
            dh[:] = inh[T.parent[level]]
            Dh.append(dh)
        return Dh

    return DT, inherit(TT, DT), DS, inherit(TS, DS), cdir
