"""Oct-based AMR hierarchies on the unit box.

Level ``l`` has cells of size ``2**-l``; a cell index ``(i, j, k)`` lies in
``[0, 2**l)^3``.  An oct at level ``l`` is a 2x2x2 block of level-``l`` cells
and is named by its coordinates ``(I, J, K) = (i >> 1, j >> 1, k >> 1)``, which
is also the index of its parent cell at level ``l - 1`` (the oct tree of the
paper, Fig. 1).  The base level covers the whole box.

Balance rule (neighbours only at ``l - 1``, ``l``, ``l + 1``, Sect. 3.1): an oct
at level ``l`` may exist only if every face neighbour of its parent cell exists
at level ``l - 1`` or lies outside the box.  The generators below only refine a
cell whose six face neighbours exist at its own level, which keeps that rule.

Oct lists are returned in a seeded random order so that no consumer can rely on
the order in which they are listed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_FACE_OFFSETS = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]],
                         dtype=np.int64)
_CHILD_OFFSETS = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=np.int64)


@dataclass
class Hierarchy:
    base_level: int
    octs: dict = field(default_factory=dict)  # level -> int32 array (n_oct, 3)

    @property
    def max_level(self) -> int:
        return max(self.octs)

    @property
    def levels(self):
        return list(range(self.base_level, self.max_level + 1))

    def n_slots(self, level: int) -> int:
        return 8 * len(self.octs[level])

    def total_slots(self) -> int:
        return sum(self.n_slots(l) for l in self.levels)


def _keys(ijk: np.ndarray, level: int) -> np.ndarray:
    n = np.int64(1) << level
    ijk = ijk.astype(np.int64)
    return (ijk[:, 0] * n + ijk[:, 1]) * n + ijk[:, 2]


def cell_coords_of_octs(octs: np.ndarray) -> np.ndarray:
    """Cell indices of all 8 children of each oct, oct-major, x fastest within an oct."""
    octs = np.asarray(octs, dtype=np.int64)
    return (2 * octs[:, None, :] + _CHILD_OFFSETS[None, :, :]).reshape(-1, 3)


def _full_octs(level: int) -> np.ndarray:
    n = 1 << (level - 1)
    g = np.arange(n, dtype=np.int32)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)


def _shuffled(arr: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    return np.ascontiguousarray(arr[rng.permutation(len(arr))].astype(np.int32))


def _slot_keys(h: Hierarchy, level: int) -> np.ndarray:
    return np.sort(_keys(cell_coords_of_octs(h.octs[level]), level))


def _exists(sorted_keys: np.ndarray, ijk: np.ndarray, level: int) -> np.ndarray:
    k = _keys(ijk, level)
    pos = np.searchsorted(sorted_keys, k)
    pos = np.minimum(pos, len(sorted_keys) - 1)
    return sorted_keys[pos] == k


def _eligible(h: Hierarchy, level: int, cells: np.ndarray) -> np.ndarray:
    """Cells whose six face neighbours exist at ``level`` or are outside the box."""
    n = 1 << level
    skeys = _slot_keys(h, level)
    ok = np.ones(len(cells), dtype=bool)
    for off in _FACE_OFFSETS:
        nb = cells.astype(np.int64) + off
        inside = np.all((nb >= 0) & (nb < n), axis=1)
        ex = np.zeros(len(cells), dtype=bool)
        if inside.any():
            ex[inside] = _exists(skeys, nb[inside], level)
        ok &= (~inside) | ex
    return ok


def _eligible_octwise(h: Hierarchy, level: int) -> np.ndarray:
    """``_eligible`` for all cells of ``level`` in ``cell_coords_of_octs`` order: a face
    neighbour outside a cell's oct lies in the neighbouring oct, so one lookup per oct
    and face decides it for the cells on that side."""
    octs = np.asarray(h.octs[level], dtype=np.int64)
    m = 1 << (level - 1)
    okeys = np.sort(_keys(octs, level - 1))
    ok = np.ones((len(octs), 8), dtype=bool)
    pos = np.arange(8)
    for d, off in enumerate(_FACE_OFFSETS):
        axis, plus = d // 2, d % 2
        nb = octs + off
        inside = (nb[:, axis] >= 0) & (nb[:, axis] < m)
        nb_ok = ~inside
        if inside.any():
            nb_ok[inside] = _exists(okeys, nb[inside], level - 1)
        outer = ((pos >> axis) & 1) == plus  # cells whose face in this direction leaves the oct
        ok[:, outer] &= nb_ok[:, None]
    return ok.reshape(-1)


def uniform_hierarchy(level: int, seed: int = 0) -> Hierarchy:
    rng = np.random.default_rng(seed)
    return Hierarchy(level, {level: _shuffled(_full_octs(level), rng)})


def centred_box_hierarchy(base_level: int, lo: int, hi: int, seed: int = 0) -> Hierarchy:
    """Base level plus one finer level refining the coarse cells ``lo..hi-1`` per axis."""
    rng = np.random.default_rng(seed)
    g = np.arange(lo, hi, dtype=np.int32)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    fine = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    return Hierarchy(base_level, {base_level: _shuffled(_full_octs(base_level), rng),
                                  base_level + 1: _shuffled(fine, rng)})


def random_balanced_hierarchy(seed: int, base_level: int, max_level: int, p_refine: float = 0.3,
                              blob: bool = True) -> Hierarchy:
    """Random balanced hierarchy.  With ``blob`` the refinement probability is higher
    near a random centre, which yields nested, irregular refined regions."""
    rng = np.random.default_rng(seed)
    h = Hierarchy(base_level, {base_level: _shuffled(_full_octs(base_level), rng)})
    centre = rng.uniform(0.25, 0.75, size=3)
    for level in range(base_level, max_level):
        cells = cell_coords_of_octs(h.octs[level])
        elig = _eligible(h, level, cells)
        x = (cells + 0.5) / (1 << level)
        if blob:
            d = np.linalg.norm(x - centre, axis=1)
            prob = p_refine * np.exp(-(d / 0.3) ** 2) * 2.0
        else:
            prob = np.full(len(cells), p_refine)
        pick = elig & (rng.uniform(size=len(cells)) < prob)
        if not pick.any():
            break
        h.octs[level + 1] = _shuffled(cells[pick], rng)
    return h


def budgeted_hierarchy(base_level: int, max_level: int, criterion, threshold: float, quota: int,
                       seed: int = 0):
    """Refine, level by level, the eligible cells with the largest criterion above
    ``threshold``, at most ``quota`` cells per level; ties are broken by cell key.

    ``criterion(level, cells) -> float array``.  Returns the hierarchy and the
    number of refined cells per level.
    """
    rng = np.random.default_rng(seed)
    h = Hierarchy(base_level, {base_level: _shuffled(_full_octs(base_level), rng)})
    counts = {}
    for level in range(base_level, max_level):
        cells = cell_coords_of_octs(h.octs[level])
        elig = _eligible_octwise(h, level)
        crit = np.asarray(criterion(level, cells), dtype=np.float64)
        cand = np.nonzero(elig & (crit > threshold))[0]
        order = np.lexsort((_keys(cells[cand], level), -crit[cand]))
        chosen = cand[order[:quota]]
        counts[level] = len(chosen)
        if len(chosen) == 0:
            break
        h.octs[level + 1] = _shuffled(cells[chosen], rng)
    return h, counts


def is_balanced(h: Hierarchy) -> bool:
    """Check the balance rule and that every oct has an existing parent."""
    for level in h.levels:
        octs = h.octs[level].astype(np.int64)
        if level == h.base_level:
            if len(octs) != (1 << (level - 1)) ** 3:
                return False
            continue
        parent_keys = _slot_keys(h, level - 1)
        if not _exists(parent_keys, octs, level - 1).all():
            return False
        n = 1 << (level - 1)
        for off in _FACE_OFFSETS:
            nb = octs + off
            inside = np.all((nb >= 0) & (nb < n), axis=1)
            if inside.any() and not _exists(parent_keys, nb[inside], level - 1).all():
                return False
    return True
