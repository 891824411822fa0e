"""Oracle: mesh connectivity, validation and space-filling-curve renumbering.

Test infrastructure only (see the package docstring).

Connectivity follows the finite-volume setting of Sec. 2 (a polygon cell
bounded by its straight faces, eq. (semidiscrete)): face k of a cell runs
from its vertex k to vertex k+1 (counter-clockwise), and the neighbour across
it is the unique other cell owning the same edge in the opposite direction.
Periodic domains identify seam nodes through canonical node ids; the periodic
shift of a face is the exact offset that moves the neighbour next to the cell.

The renumbering is not part of the paper; it fixes the library's internal
cell order: quadrilaterals first, then triangles, each group sorted by the
order-16 Hilbert index of the cell's vertex average, ties by original id.
"""
from __future__ import annotations

import dataclasses

import numpy as np


class MeshError(ValueError):
    pass


@dataclasses.dataclass
class Conn:
    nf: np.ndarray         # int32 [N]   faces per cell (3 or 4)
    nbr: np.ndarray        # int64 [N,4] neighbour across face k, -1 = boundary / unused
    nbr_face: np.ndarray   # int64 [N,4] the neighbour's face index of the shared edge
    shift: np.ndarray      # f64  [N,4,2] add to the neighbour's coordinates
    area: np.ndarray       # f64  [N] shoelace area (validation only)


def _shoelace(xy, cells, nf):
    a = np.zeros(cells.shape[0])
    for k in range(4):
        kn = np.where(k + 1 < nf, k + 1, 0)
        ok = k < nf
        p = xy[np.maximum(cells[:, k], 0)]
        q = xy[np.maximum(np.take_along_axis(cells, kn[:, None], 1)[:, 0], 0)]
        a += np.where(ok, p[:, 0] * q[:, 1] - q[:, 0] * p[:, 1], 0.0)
    return 0.5 * a


def connectivity(mesh) -> Conn:
    """Face neighbours, neighbour face index and periodic shift of every face.

    Raises MeshError for: a cell whose node count is not 3 or 4, an invalid
    node index, repeated nodes in a cell, non-positive signed area, an edge
    owned by more than two cells, two owners traversing an edge in the same
    direction, or an unmatched face on a periodic mesh.
    """
    cells = np.asarray(mesh.cell_nodes, dtype=np.int64)
    xy = np.asarray(mesh.node_xy, dtype=np.float64)
    n = cells.shape[0]
    nn = xy.shape[0]
    if cells.ndim != 2 or cells.shape[1] != 4:
        raise MeshError("cell_nodes must be [n_cells, 4]")
    if (cells[:, :3] < 0).any() or (cells >= nn).any() or (cells[:, 3] < -1).any():
        raise MeshError("invalid node index")
    nf = np.where(cells[:, 3] < 0, 3, 4).astype(np.int32)
    for i in range(4):
        for j in range(i + 1, 4):
            same = (cells[:, i] == cells[:, j]) & (j < nf)
            if same.any():
                raise MeshError("repeated node in a cell")
    area = _shoelace(xy, cells, nf)
    if not (area > 0).all():
        raise MeshError("cell with non-positive signed area (not counter-clockwise)")
    canon = np.arange(nn, dtype=np.int64) if mesh.node_id is None else \
        np.asarray(mesh.node_id, dtype=np.int64)

    # all half-edges (cell, face k) with k < nf
    cid = np.repeat(np.arange(n), 4)
    kid = np.tile(np.arange(4), n)
    keep = kid < nf[cid]
    cid, kid = cid[keep], kid[keep]
    kn = np.where(kid + 1 < nf[cid], kid + 1, 0)
    a = cells[cid, kid]
    b = cells[cid, kn]
    ca, cb = canon[a], canon[b]
    lo, hi = np.minimum(ca, cb), np.maximum(ca, cb)
    if (lo == hi).any():
        raise MeshError("degenerate edge (both ends identified)")
    m = int(canon.max()) + 1
    key = lo * m + hi
    order = np.argsort(key, kind="stable")
    ks = key[order]
    uniq, start, counts = np.unique(ks, return_index=True, return_counts=True)
    if (counts > 2).any():
        raise MeshError("edge shared by more than two cells")
    nbr = np.full((n, 4), -1, dtype=np.int64)
    nbr_face = np.full((n, 4), -1, dtype=np.int64)
    shift = np.zeros((n, 4, 2))
    pair = counts == 2
    h1 = order[start[pair]]
    h2 = order[start[pair] + 1]
    if (ca[h1] != cb[h2]).any() or (cb[h1] != ca[h2]).any():
        raise MeshError("edge traversed in the same direction by both owners")
    for x, y in ((h1, h2), (h2, h1)):
        nbr[cid[x], kid[x]] = cid[y]
        nbr_face[cid[x], kid[x]] = kid[y]
        # node a[x] and node b[y] are the same canonical node
        shift[cid[x], kid[x]] = xy[a[x]] - xy[b[y]]
    if mesh.bc == "periodic" and (~pair).any():
        raise MeshError("unmatched face on a periodic mesh")
    return Conn(nf=nf, nbr=nbr, nbr_face=nbr_face, shift=shift, area=area)


# --------------------------------------------------------------------------
# space-filling curve
# --------------------------------------------------------------------------

def hilbert_index(qx, qy, order: int = 16):
    """Index along the Hilbert curve of the 2^order x 2^order grid.

    Recursive definition: the square is split into four quadrants visited in
    the order (0,0), (0,1), (1,1), (1,0) (x, y); the curve inside quadrant
    (0,0) is the parent curve transposed, inside (1,0) anti-transposed, and
    inside the two upper quadrants it is the parent curve itself."""
    x = np.asarray(qx, dtype=np.int64).copy()
    y = np.asarray(qy, dtype=np.int64).copy()
    d = np.zeros_like(x)
    s = 1 << (order - 1)
    while s >= 1:
        rx = (x >= s).astype(np.int64)
        ry = (y >= s).astype(np.int64)
        quadrant = np.where(rx == 0, np.where(ry == 0, 0, 1), np.where(ry == 1, 2, 3))
        d += quadrant * s * s
        lx = x - rx * s
        ly = y - ry * s
        tx = np.where(quadrant == 0, ly, np.where(quadrant == 3, s - 1 - ly, lx))
        ty = np.where(quadrant == 0, lx, np.where(quadrant == 3, s - 1 - lx, ly))
        x, y = tx, ty
        s >>= 1
    return d


def sfc_keys(mesh):
    """Quantised vertex average of each cell and its Hilbert index.

    The vertex average is (x_0 + x_1 + ... ) / n summed in vertex order; the
    quantisation is q = min(65535, floor(65536 (c - lo) / (hi - lo))) with lo,
    hi the bounding box of all nodes."""
    cells = np.asarray(mesh.cell_nodes, dtype=np.int64)
    xy = np.asarray(mesh.node_xy, dtype=np.float64)
    nf = np.where(cells[:, 3] < 0, 3, 4)
    p = xy[np.maximum(cells, 0)]
    sx = p[:, 0, 0] + p[:, 1, 0]
    sx = sx + p[:, 2, 0]
    sy = p[:, 0, 1] + p[:, 1, 1]
    sy = sy + p[:, 2, 1]
    sx = np.where(nf == 4, sx + p[:, 3, 0], sx)
    sy = np.where(nf == 4, sy + p[:, 3, 1], sy)
    cx = sx / nf
    cy = sy / nf
    lo = xy.min(axis=0)
    hi = xy.max(axis=0)
    qx = np.minimum(65535, np.floor(65536.0 * (cx - lo[0]) / (hi[0] - lo[0]))).astype(np.int64)
    qy = np.minimum(65535, np.floor(65536.0 * (cy - lo[1]) / (hi[1] - lo[1]))).astype(np.int64)
    return hilbert_index(qx, qy, 16)


def sfc_permutation(mesh):
    """Returns (new_of_old, old_of_new): quadrilaterals first, then
    triangles, each by (Hilbert index, original id)."""
    cells = np.asarray(mesh.cell_nodes)
    n = cells.shape[0]
    is_tri = (cells[:, 3] < 0).astype(np.int64)
    d = sfc_keys(mesh)
    old_of_new = np.lexsort((np.arange(n), d, is_tri))
    new_of_old = np.empty(n, dtype=np.int64)
    new_of_old[old_of_new] = np.arange(n)
    return new_of_old, old_of_new
