"""Fast directional matrix-vector multiplication (Sect. 2.6, Alg. 4).  Oracle.

``build`` assembles what Alg. 4 takes as input: the two box cluster trees
(Alg. 1), the block tree (Alg. 2), the direction sets (Alg. 3) and the active
and inherited directions ``D(t), D^(t), D(s), D^(s)`` (Sect. 2.6).  ``matvec``
then runs Alg. 4 in the paper's order, in FP64 / complex128:

1. ``g = 0``;
2. S2M: ``v~_{s,c} = L_{s,c}^* v|_s`` for leaves ``s``, ``c in D(s) u D^(s)``;
3. M2M, levels ``p-1 .. 0``: ``v~_{s,c} = sum_{s'} E_{s',c}^* v~_{s',c'}``,
   ``c' = dir_(l+1)(c)``;
4. M2L: ``g~_{t,c} += A_{c,t x s} v~_{s,c}`` over admissible leaves;
5. L2L, levels ``0 .. p-1``: ``g~_{t',c'} += E_{t',c} g~_{t,c}``;
6. L2T: ``g|_t += L_{t,c} g~_{t,c}`` for leaves ``t``;
7. near field: ``g|_t += A|_{t x s} v|_s`` over inadmissible leaves.

Steps use the paper's absolute plane-wave factors ``exp(i kappa <x, c>)``
(eq. of ``L_{t,c,nu}``) and the transfer matrices of Sect. 2.5.  Blocks of
step 4 that share a level and an offset are applied as one matrix product
(Sect. 2.7 stores their coupling matrix once); this only changes the order
of the sums.

``sample_rows`` runs the same algorithm for a few target rows: the block tree
is restricted to the ancestors of those rows' leaves (so only the moments they
need are formed), and L2T / near field are evaluated at those rows only.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import emulate, lowrank
from .tree import BoxTree, build_box_tree
from .partition import ETA2, BlockTree, block_tree
from .directions import DirectionSets, active_directions, high_frequency_level
from .interpolation import (coupling_matrix, directional_part, helmholtz,
                            interpolation_rows, transfer_reference)


@dataclass
class Plan:
    TT: BoxTree
    TS: BoxTree
    BT: BlockTree
    dirs: DirectionSets
    kappa: float
    m: int
    l_hf: int
    eta2: float
    DT: list
    DhT: list
    DS: list
    DhS: list
    cdir: list
    rows: np.ndarray | None = None  # sampled target rows (user indices)
    timings: dict = field(default_factory=dict)
    debug: dict = field(default_factory=dict)

    @property
    def levels(self) -> int:
        return self.TT.levels

    @property
    def K(self) -> int:
        return (self.m + 1) ** 3

    def side(self, level: int) -> np.ndarray:
        return self.TT.side(level)


def _validate(box, kappa, levels, m):
    lo = np.asarray(box[:3], dtype=np.float64)
    hi = np.asarray(box[3:], dtype=np.float64)
    if not (np.all(np.isfinite(lo)) and np.all(np.isfinite(hi)) and
            np.all(hi > lo)):
        raise ValueError("invalid root box")
    side = hi - lo
    if not (np.isfinite(kappa) and kappa >= 0):
        raise ValueError("kappa must be finite and >= 0")
    if not (0 <= levels <= 10):
        raise ValueError("levels must be in [0, 10]")
    if not (1 <= m <= 8):
        raise ValueError("m must be in [1, 8]")
    return side


def build(points_T, points_S, kappa, box, levels, m, l_hf=None,
          eta2=ETA2, rows=None, n_max=None) -> Plan:
    """Trees (Alg. 1; ``n_max=None``: uniform to depth ``levels``, else
    adaptive with at most ``n_max`` points per leaf above that depth), block
    tree (Alg. 2), directions (Alg. 3).  ``rows``: keep only what the given
    target rows (user indices) need."""
    side = _validate(box, kappa, levels, m)
    if n_max is not None and not (int(n_max) == n_max and n_max >= 0):
        raise ValueError("n_max must be a non-negative integer")
    TT = build_box_tree(points_T, box, levels, n_max)
    TS = build_box_tree(points_S, box, levels, n_max)
    if l_hf is None:  # (the longest side for a non-cubic box)
        l_hf = high_frequency_level(kappa, float(np.max(side)), levels)
    dirs = DirectionSets(l_hf, levels)
    filt = None
    if rows is not None:
        rows = np.asarray(rows, dtype=np.int64)
        inv = np.empty(TT.n, dtype=np.int64)
        inv[TT.perm] = np.arange(TT.n)
        filt = []
        for level in range(levels + 1):  # boxes holding a requested row
            b = TT.box_of_slots(level, inv[rows])
            mask = np.zeros(TT.keys[level].shape[0], dtype=bool)
            mask[b[b >= 0]] = True
            filt.append(mask)
    BT = block_tree(TT, TS, kappa, eta2, filt)
    DT, DhT, DS, DhS, cdir = active_directions(TT, TS, BT, dirs, side)
    return Plan(TT, TS, BT, dirs, float(kappa), m, l_hf, eta2,
                DT, DhT, DS, DhS, cdir, rows)


def apply_coupling(m, h, o, kappa, c, M, m2l="fp64"):
    """One group of the coupling step: every admissible block of one level
    and offset ``o`` shares ``A_{c,t x s}`` (Sect. 2.7); rows of ``M`` are the
    blocks' source moments, the result rows their contributions to the
    target locals.  ``m2l = "aca:<eps>"`` applies the matrix compressed by
    adaptive cross approximation to tolerance eps (Sect. 2.7), A ~ U W^*."""
    A = coupling_matrix(m, h, o, kappa, c)
    if m2l.startswith("aca:"):
        U, W = lowrank.aca_dense(A, float(m2l[4:]))
        return (M @ W.conj()) @ U.T
    return emulate.product(A, M, m2l)


def _segments(start, count):
    """Tree slots of boxes given their ranges, plus each slot's box."""
    total = int(count.sum())
    box = np.repeat(np.arange(start.shape[0]), count)
    first = np.concatenate(([0], np.cumsum(count)[:-1]))
    slots = np.repeat(start, count) + (np.arange(total) - np.repeat(first, count))
    return slots, box


def _chunks(counts, limit):
    """Split consecutive boxes into chunks of at most ~limit points."""
    out, acc, begin = [], 0, 0
    for i, c in enumerate(counts):
        if acc + c > limit and i > begin:
            out.append((begin, i))
            begin, acc = i, 0
        acc += int(c)
    if begin < len(counts):
        out.append((begin, len(counts)))
    return out


def _widen(x: np.ndarray) -> np.ndarray:
    """``x`` as complex128; zero rows are not copied (so that a large array
    whose pages were never written stays unbacked)."""
    if x.dtype == np.complex128:
        return x
    y = np.zeros(x.shape, dtype=np.complex128)
    nz = np.flatnonzero(np.any(x != 0, axis=tuple(range(1, x.ndim))))
    y[nz] = x[nz]
    return y


def _coupling_level(plan: Plan, level: int, mom_level, loc_level, m2l: str):
    """Step 4 of Alg. 4 on one level: every admissible block (t, s) of the
    level adds ``A_{c, t x s} v~_{s,c}`` to ``g~_{t,c}``, blocks grouped by
    offset (Sect. 2.7), groups in ascending offset order."""
    TT, TS, BT, dirs = plan.TT, plan.TS, plan.BT, plan.dirs
    t, s = BT.adm_t[level], BT.adm_s[level]
    if t.size == 0:
        return
    o = TT.coords[level][t] - TS.coords[level][s]
    c = plan.cdir[level]
    cv = dirs.vectors(level)
    h = plan.side(level)
    uo, inv = np.unique(o, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    order = np.argsort(inv, kind="stable")
    bounds = np.concatenate(([0], np.cumsum(np.bincount(inv, minlength=uo.shape[0]))))
    for gi in range(uo.shape[0]):
        idx = order[bounds[gi]:bounds[gi + 1]]
        cg = c[idx[0]]
        loc_level[t[idx], cg] += apply_coupling(plan.m, h, uo[gi], plan.kappa, cv[cg],
                                                mom_level[s[idx], cg], m2l)


def matvec(plan: Plan, v, chunk_points: int = 65536, keep: bool = False,
           m2l="fp64", chunk_boxes: int = 8192):
    """Alg. 4: ``g ~= A v`` in the user's target order (complex128).

    ``m2l`` other than ``"fp64"`` emulates a reduced-precision coupling step
    (see ``oracle.emulate``) or, as ``"aca:<eps>"``, applies the coupling
    matrices compressed by ACA (``oracle.lowrank``); the default is the
    plain FP64 algorithm.  A sequence of such modes returns one result per
    mode, sharing the forward transformation (steps 1-3).

    Memory: the coupling step of a level runs as soon as that level's
    moments exist, and the moments of a level are dropped once its coupling
    step and its parents' M2M have read them (``keep`` holds them all).
    Each level's coupling step reads only its own moments and writes only
    its own locals, which the backward transformation reads after every
    coupling step has run, so this is the same arithmetic in the same order
    as running all of step 3 before all of step 4.  M2M and L2L take the
    boxes ``chunk_boxes`` parents at a time (per-parent sums unchanged).
    """
    single = isinstance(m2l, str)
    modes = [m2l] if single else list(m2l)
    t0 = time.perf_counter()
    TT, TS, BT, dirs = plan.TT, plan.TS, plan.BT, plan.dirs
    p, m, K, kappa = plan.levels, plan.m, plan.K, plan.kappa
    v = np.asarray(v, dtype=np.complex128).reshape(-1)
    if v.shape[0] != TS.n:
        raise ValueError("v has the wrong length")
    if TT.n == 0 or TS.n == 0:
        z = np.zeros(TT.n, dtype=np.complex128) if plan.rows is None \
            else np.zeros(plan.rows.shape[0], dtype=np.complex128)
        return z if single else [z.copy() for _ in modes]
    vt = v[TS.perm]
    Eref = transfer_reference(m)
    loc = {mode: [np.zeros((plan.DT[l] | plan.DhT[l]).shape + (K,),
                           dtype=emulate.accumulate_dtype(mode)) for l in range(p + 1)]
           for mode in modes}
    t_m2l = 0.0

    def s2m(level):
        """S2M for the leaves of T_S on ``level``."""
        need = (plan.DS[level] | plan.DhS[level]) & TS.is_leaf(level)[:, None]
        cvec = dirs.vectors(level)
        for c in range(need.shape[1]):
            leaves = np.flatnonzero(need[:, c])
            for a, b in _chunks(TS.count[level][leaves], chunk_points):
                lv = leaves[a:b]
                slots, owner = _segments(TS.start[level][lv], TS.count[level][lv])
                y = TS.points[slots]
                L = interpolation_rows(y, TS.lo[level][lv][owner], TS.hi[level][lv][owner], m)
                # conj(L_{s,c}) rows times v: L_{s,nu}(y) exp(-i kappa <y,c>) v
                w = np.exp(-1j * kappa * (y @ cvec[c])) * vt[slots]
                contrib = L * w[:, None]
                seg = np.concatenate(([0], np.cumsum(TS.count[level][lv])[:-1]))
                mom[level][lv, c] = np.add.reduceat(contrib, seg, axis=0)

    # --- S2M (leaves of T_S on the last level; other levels' leaves below) -
    mom = [None] * (p + 1)
    mom[p] = np.zeros((plan.DS[p] | plan.DhS[p]).shape + (K,), dtype=np.complex128)
    s2m(p)
    plan.timings["s2m"] = time.perf_counter() - t0

    # --- M2M (levels p-1 .. 0), each level's coupling step once its moments
    # --- exist (step 4 per level; see the docstring) -------------------------
    t1 = time.perf_counter()
    for level in range(p - 1, -1, -1):
        need = plan.DS[level] | plan.DhS[level]
        mom[level] = np.zeros(need.shape + (K,), dtype=np.complex128)
        if need.any():
            par_dir = dirs.parent_index(level)
            cv, cv1 = dirs.vectors(level), dirs.vectors(level + 1)
            for c in range(need.shape[1]):
                all_parents = np.flatnonzero(need[:, c] & ~TS.is_leaf(level))
                cp = par_dir[c]
                for a in range(0, all_parents.size, chunk_boxes):
                    parents = all_parents[a:a + chunk_boxes]
                    ch, owner = _segments(TS.child_start[level][parents],
                                          TS.child_count[level][parents])
                    Ed = directional_part(TS.lo[level + 1][ch], TS.hi[level + 1][ch],
                                          m, kappa, cv[c], cv1[cp])
                    w = np.conj(Ed) * mom[level + 1][ch, cp]  # (E^d)^* v~_{s',c'}
                    octant = TS.keys[level + 1][ch] & 7
                    contrib = np.empty_like(w)
                    for q in range(8):
                        sel = octant == q
                        if sel.any():
                            contrib[sel] = w[sel] @ Eref[q]  # rows of E_{s'}^T w
                    seg = np.concatenate(([0], np.cumsum(TS.child_count[level][parents])[:-1]))
                    mom[level][parents, c] = np.add.reduceat(contrib, seg, axis=0)
            s2m(level)  # leaves of this level (adaptive trees)
        t2 = time.perf_counter()
        for mode in modes:
            _coupling_level(plan, level + 1, mom[level + 1], loc[mode][level + 1], mode)
        t_m2l += time.perf_counter() - t2
        if not keep:
            mom[level + 1] = None
    t2 = time.perf_counter()
    for mode in modes:
        _coupling_level(plan, 0, mom[0], loc[mode][0], mode)
    t_m2l += time.perf_counter() - t2
    if not keep:
        mom[0] = None
    plan.timings["m2l"] = t_m2l
    plan.timings["m2m"] = time.perf_counter() - t1 - t_m2l
    for mode in modes:
        loc[mode] = [_widen(x) for x in loc[mode]]

    if plan.rows is not None:
        inv = np.empty(TT.n, dtype=np.int64)
        inv[TT.perm] = np.arange(TT.n)
        want = np.zeros(TT.n, dtype=bool)
        want[inv[plan.rows]] = True
    results = []
    for mode in modes:
        lm = loc[mode]
        # --- L2L (levels 0 .. p-1) -----------------------------------------
        t3 = time.perf_counter()
        for level in range(p):
            need = plan.DT[level] | plan.DhT[level]
            if not need.any():
                continue
            par_dir = dirs.parent_index(level)
            cv, cv1 = dirs.vectors(level), dirs.vectors(level + 1)
            for c in range(need.shape[1]):
                all_parents = np.flatnonzero(need[:, c] & ~TT.is_leaf(level))
                cp = par_dir[c]
                for a in range(0, all_parents.size, chunk_boxes):
                    parents = all_parents[a:a + chunk_boxes]
                    ch, owner = _segments(TT.child_start[level][parents],
                                          TT.child_count[level][parents])
                    gpar = lm[level][parents[owner], c]
                    octant = TT.keys[level + 1][ch] & 7
                    Eg = np.empty_like(gpar)
                    for q in range(8):
                        sel = octant == q
                        if sel.any():
                            Eg[sel] = gpar[sel] @ Eref[q].T  # rows of E_{t'} g
                    Ed = directional_part(TT.lo[level + 1][ch], TT.hi[level + 1][ch],
                                          m, kappa, cv[c], cv1[cp])
                    lm[level + 1][ch, cp] += Ed * Eg
        plan.timings["l2l"] = time.perf_counter() - t3

        # --- L2T (leaves of T_T, last level first) -------------------------
        t4 = time.perf_counter()
        g_tree = np.zeros(TT.n, dtype=np.complex128)
        for lev in [p] + list(range(p)):
            need = (plan.DT[lev] | plan.DhT[lev]) & TT.is_leaf(lev)[:, None]
            cvec = dirs.vectors(lev)
            for c in range(need.shape[1]):
                leaves = np.flatnonzero(need[:, c])
                for a, b in _chunks(TT.count[lev][leaves], chunk_points):
                    lv = leaves[a:b]
                    slots, owner = _segments(TT.start[lev][lv], TT.count[lev][lv])
                    if plan.rows is not None:
                        sel = want[slots]
                        slots, owner = slots[sel], owner[sel]
                    x = TT.points[slots]
                    L = interpolation_rows(x, TT.lo[lev][lv][owner], TT.hi[lev][lv][owner], m)
                    ph = np.exp(1j * kappa * (x @ cvec[c]))
                    g_tree[slots] += ph * np.einsum("nk,nk->n", L, lm[lev][lv[owner], c])
        plan.timings["l2t"] = time.perf_counter() - t4

        # --- near field (inadmissible leaf blocks, last level first) ---------
        t5 = time.perf_counter()
        for lev in [p] + list(range(p)):
            nt, ns = BT.near_t[lev], BT.near_s[lev]
            if not nt.size:
                continue
            tslots, towner = _segments(TT.start[lev][nt], TT.count[lev][nt])
            if plan.rows is not None:
                sel = want[tslots]
                tslots, towner = tslots[sel], towner[sel]
            # every target slot meets every source slot of its pair's source box
            srcs = ns[towner]
            cnt = TS.count[lev][srcs]
            for a, b in _chunks(cnt, 4 * chunk_points):
                ts = tslots[a:b]
                sl, own = _segments(TS.start[lev][srcs[a:b]], cnt[a:b])
                tj = ts[own]
                d = TT.points[tj] - TS.points[sl]
                # f(x, y) = 0 exactly when the two points coincide (diagonal)
                same = np.all(TT.points[tj] == TS.points[sl], axis=1)
                r = np.sqrt(np.sum(d * d, axis=1))
                r[same] = 0.0
                np.add.at(g_tree, tj, helmholtz(r, kappa) * vt[sl])
        plan.timings["near"] = time.perf_counter() - t5

        g = np.zeros(TT.n, dtype=np.complex128)
        g[TT.perm] = g_tree
        results.append(g[plan.rows] if plan.rows is not None else g)
    plan.timings["total"] = time.perf_counter() - t0
    if keep:  # intermediate moments and locals (absolute phase form)
        plan.debug = {"mom": mom, "loc": loc[modes[0]]}
    return results[0] if single else results


def sample_rows(points_T, points_S, v, kappa, box, levels, m, rows,
                l_hf=None, eta2=ETA2, n_max=None) -> np.ndarray:
    """Alg. 4 evaluated at the given target rows only (user indices)."""
    plan = build(points_T, points_S, kappa, box, levels, m, l_hf, eta2, rows, n_max)
    return matvec(plan, v)


def structure(plan: Plan) -> dict:
    """Canonical integer description of the plan, for structure parity.

    Keys: ``perm_T``/``perm_S``; per level ``keys_T{l}``, ``start_T{l}``,
    ``count_T{l}`` (and ``_S``); ``l_hf``; per level the number of admissible
    blocks ``nc{l}``, the distinct offsets they use ``off{l}`` (sorted, (n,3))
    with their direction index ``offdir{l}`` and use count ``offcnt{l}``;
    ``near_pairs`` and ``near_entries`` (sum of ``#t * #s`` over inadmissible
    leaves); per level the active / inherited direction sets as sorted
    ``box * ndir + dir`` codes ``D_T{l}``, ``Dh_T{l}``, ``D_S{l}``, ``Dh_S{l}``.
    """
    out = {"perm_T": plan.TT.perm, "perm_S": plan.TS.perm,
           "l_hf": np.array([plan.l_hf])}
    p = plan.levels
    for tag, T in (("T", plan.TT), ("S", plan.TS)):
        for l in range(p + 1):
            out[f"keys_{tag}{l}"] = T.keys[l]
            out[f"start_{tag}{l}"] = T.start[l]
            out[f"count_{tag}{l}"] = T.count[l]
    for l in range(p + 1):
        t, s = plan.BT.adm_t[l], plan.BT.adm_s[l]
        out[f"nc{l}"] = np.array([t.shape[0]])
        if t.size:
            o = plan.TT.coords[l][t] - plan.TS.coords[l][s]
            uo, first, cnt = np.unique(o, axis=0, return_index=True,
                                       return_counts=True)
            out[f"off{l}"] = uo
            out[f"offdir{l}"] = plan.cdir[l][first]
            out[f"offcnt{l}"] = cnt
        else:
            out[f"off{l}"] = np.zeros((0, 3), dtype=np.int64)
            out[f"offdir{l}"] = np.zeros(0, dtype=np.int64)
            out[f"offcnt{l}"] = np.zeros(0, dtype=np.int64)
        for tag, D in (("D_T", plan.DT), ("Dh_T", plan.DhT), ("D_S", plan.DS),
                       ("Dh_S", plan.DhS)):
            b, c = np.nonzero(D[l])
            out[f"{tag}{l}"] = np.sort(b * D[l].shape[1] + c)
    pairs = entries = 0
    for l in range(p + 1):  # inadmissible leaf blocks of every level
        nt, ns = plan.BT.near_t[l], plan.BT.near_s[l]
        pairs += nt.shape[0]
        entries += int(np.sum(plan.TT.count[l][nt] * plan.TS.count[l][ns]))
    out["near_pairs"] = np.array([pairs])
    out["near_entries"] = np.array([entries])
    return out
