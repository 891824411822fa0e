"""Oracle: big-stencil slot selection and candidate sub-stencils.

Test infrastructure only (see the package docstring).

Paper: Sec. 3.1 (quadrilateral stencil, its selection procedure with the
presence flags E_j and the substitutions i_j -> i_0 and i_j -> i_{j-4}; the
twelve sub-stencils S_1..S_12) and Sec. 3.2 (triangular stencil, the
substitutions i_j -> i_0 and i_j -> i_{j-3}; the nine sub-stencils S_1..S_9).

Reading of the geometry (the stencil figures of the paper are not
available): with vertices v_0..v_{n-1} counter-clockwise, face k runs from
v_k to v_{k+1} and i_{k+1} is the neighbour across it.  An outer slot is
``slot(c, v)``: the cell across the face of face-neighbour c that contains
vertex v and is not the face c shares with i_0.  The slot table below makes
every substitution a fallback to a cell at the same vertex, and keeps the
printed sub-stencils (S_5 = {i0, i1, i5} etc.) made of cells that touch.

An outer slot is *absent* (E_j = 0) when there is no such cell (a boundary,
or a ghost face neighbour), when it is i_0 or one of the face neighbours, or
when it repeats an earlier present slot (slot-index order).  Cells are
compared together with their periodic image (id and shift).  An absent slot
takes the cell of its replacement, recursively.

Transmissive boundary faces: the face neighbour is a ghost, the mirror image
of i_0 across the face line, carrying the value of i_0 and present (E = 1);
slots reached through a ghost are absent.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class TypeSpec:
    n: int                      # faces
    S: int                      # big-stencil size (slots 0..S-1)
    M: int                      # candidate sub-stencils
    outer: tuple                # for slots n+1..S-1: (face k, 0 = first vertex v_k, 1 = second v_{k+1})
    replace: tuple              # replacement slot of each outer slot
    sub: tuple                  # (a, b) slots of S_j = {i0, a, b}, j = 1..M
    d_pairs: tuple              # optimisation: slot -> candidate(s) whose |gamma| sets d


# Sec. 3.1: S1={i0,i1,i2} S2={i0,i2,i3} S3={i0,i3,i4} S4={i0,i4,i1} S5={i0,i1,i5}
# S6={i0,i1,i6} S7={i0,i3,i7} S8={i0,i3,i8} S9={i0,i4,i9} S10={i0,i2,i10}
# S11={i0,i2,i11} S12={i0,i4,i12}; i5..i8 -> i0 and i9..i12 -> i_{j-4};
# optimisation weights d_j = 1/max(1,|gamma_j|) for j = 5..12.
QUAD = TypeSpec(
    n=4, S=13, M=12,
    outer=((0, 0), (0, 1), (2, 0), (2, 1), (3, 1), (1, 0), (1, 1), (3, 0)),
    replace=(0, 0, 0, 0, 5, 6, 7, 8),
    sub=((1, 2), (2, 3), (3, 4), (4, 1), (1, 5), (1, 6), (3, 7), (3, 8),
         (4, 9), (2, 10), (2, 11), (4, 12)),
    d_pairs=tuple((j, (j,)) for j in range(5, 13)),
)

# Sec. 3.2: S1={i0,i1,i2} S2={i0,i2,i3} S3={i0,i3,i1} S4={i0,i1,i4} S5={i0,i2,i5}
# S6={i0,i3,i6} S7={i0,i3,i7} S8={i0,i1,i8} S9={i0,i2,i9}; i4..i6 -> i0 and
# i7..i9 -> i_{j-3}; d_j = 1/max(1,|gamma_j|,|gamma_k|) for the pairs
# (4,8), (5,9), (6,7).
TRI = TypeSpec(
    n=3, S=10, M=9,
    outer=((0, 0), (1, 0), (2, 0), (2, 1), (0, 1), (1, 1)),
    replace=(0, 0, 0, 4, 5, 6),
    sub=((1, 2), (2, 3), (3, 1), (1, 4), (2, 5), (3, 6), (3, 7), (1, 8), (2, 9)),
    d_pairs=((4, (4, 8)), (5, (5, 9)), (6, (6, 7)), (7, (7, 6)), (8, (8, 4)), (9, (9, 5))),
)


def spec_of(nf: int) -> TypeSpec:
    return QUAD if nf == 4 else TRI


@dataclasses.dataclass
class Stencils:
    cells: np.ndarray      # int64 [m] target cells of this group (original ids)
    spec: TypeSpec
    cell: np.ndarray       # int64 [m,S] cell of each slot (ghost: the target; absent: -1)
    shift: np.ndarray      # f64 [m,S,2] periodic shift of the slot's cell
    present: np.ndarray    # bool [m,S] E_j (slot 0 always present)
    ghost: np.ndarray      # int64 [m,S] face index of a ghost slot, else -1
    resolved: np.ndarray   # int64 [m,S] slot whose cell the slot uses after substitution

    @property
    def runtime_cell(self) -> np.ndarray:
        """Cell whose average each slot reads at run time (after substitution;
        a ghost reads the target cell)."""
        return np.take_along_axis(self.cell, self.resolved, axis=1)


def build_stencils(mesh, conn, nf_value: int, cells=None) -> Stencils:
    """Slot selection for all cells with ``nf_value`` faces (or the given
    subset), vectorised over cells."""
    spec = spec_of(nf_value)
    if cells is None:
        cells = np.flatnonzero(conn.nf == nf_value)
    cells = np.asarray(cells, dtype=np.int64)
    m = cells.size
    S, n = spec.S, spec.n
    cell = np.full((m, S), -1, dtype=np.int64)
    shift = np.zeros((m, S, 2))
    present = np.zeros((m, S), dtype=bool)
    ghost = np.full((m, S), -1, dtype=np.int64)
    resolved = np.tile(np.arange(S), (m, 1))

    cell[:, 0] = cells
    present[:, 0] = True
    for k in range(n):
        nb = conn.nbr[cells, k]
        is_ghost = nb < 0
        cell[:, k + 1] = np.where(is_ghost, cells, nb)
        shift[:, k + 1] = np.where(is_ghost[:, None], 0.0, conn.shift[cells, k])
        ghost[:, k + 1] = np.where(is_ghost, k, -1)
        present[:, k + 1] = True

    for s_off, (k, end) in enumerate(spec.outer):
        j = n + 1 + s_off
        c = cell[:, k + 1]
        via_ghost = ghost[:, k + 1] >= 0
        kp = conn.nbr_face[cells, k]
        nfc = conn.nf[c]
        other = np.where(end == 0, (kp + 1) % nfc, (kp - 1 + nfc) % nfc)
        other = np.where(via_ghost, 0, other)
        cand = conn.nbr[c, other]
        cshift = shift[:, k + 1] + conn.shift[c, other]
        ok = (~via_ghost) & (cand >= 0)
        # not i0 (any image with zero shift) and not a face neighbour
        same0 = (cand == cells) & (cshift == 0).all(axis=1)
        ok &= ~same0
        for f in range(1, n + 1):
            dup = (cand == cell[:, f]) & (ghost[:, f] < 0) & (cshift == shift[:, f]).all(axis=1)
            ok &= ~dup
        for jj in range(n + 1, j):
            dup = present[:, jj] & (cand == cell[:, jj]) & (cshift == shift[:, jj]).all(axis=1)
            ok &= ~dup
        cell[:, j] = np.where(ok, cand, -1)
        shift[:, j] = np.where(ok[:, None], cshift, 0.0)
        present[:, j] = ok
        rep = spec.replace[s_off]
        resolved[:, j] = np.where(ok, j, resolved[:, rep])
    return Stencils(cells=cells, spec=spec, cell=cell, shift=shift, present=present,
                    ghost=ghost, resolved=resolved)
