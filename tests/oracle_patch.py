"""The oracle's answer at a few cells of a mesh too large for it.

An RK3 step at cell i depends only on the cells within nine face-rings of i
(three stages; the residual at a cell reads the face states of the cell and
its face neighbours, whose stencils reach two rings further).  For each
sampled cell this module cuts out the cells within ``rings`` node-rings
(a superset of the face-rings), unwraps periodic seams around the sampled
cell, and runs the oracle on that patch as a stand-alone mesh with open
(transmissive) outer faces.  Cells near the patch edge see different
stencils, but none of them is within reach of the sampled cell, so its
value equals the oracle on the whole mesh (checked against the whole-mesh
oracle on meshes it can still handle).

Test infrastructure: it reads only the mesh arrays of ``workloads`` and calls
only ``oracle``.
"""
from __future__ import annotations

import numpy as np

import workloads as wl
from oracle import weights as ow
from oracle import scheme as osc

RK3_RINGS = 9


class PatchTooLarge(Exception):
    """The domain of dependence wraps around a periodic mesh."""


class NodeIncidence:
    """Cells around each canonical node (CSR), for ring expansion."""

    def __init__(self, mesh):
        cn = mesh.cell_nodes.astype(np.int64)
        if mesh.node_id is not None:
            nid = mesh.node_id.astype(np.int64)
            cn = np.where(cn >= 0, nid[np.maximum(cn, 0)], -1)
        self.canon = cn
        flat = cn.ravel()
        cells = np.repeat(np.arange(cn.shape[0], dtype=np.int64), cn.shape[1])
        keep = flat >= 0
        flat, cells = flat[keep], cells[keep]
        order = np.argsort(flat, kind="stable")
        self.cells = cells[order]
        n_nodes = int(flat.max()) + 1 if flat.size else 0
        self.start = np.zeros(n_nodes + 1, dtype=np.int64)
        np.add.at(self.start, flat + 1, 1)
        self.start = np.cumsum(self.start)

    def grow(self, cells, rings):
        cur = np.unique(np.asarray(cells, dtype=np.int64))
        for _ in range(rings):
            nodes = np.unique(self.canon[cur])
            nodes = nodes[nodes >= 0]
            a, b = self.start[nodes], self.start[nodes + 1]
            lens = b - a
            idx = np.repeat(a - np.cumsum(lens) + lens, lens) + np.arange(lens.sum())
            cur = np.union1d(cur, self.cells[idx])
        return cur


def patch_mesh(mesh, inc: NodeIncidence, centre_cell: int, rings: int):
    """The cells within ``rings`` node-rings of ``centre_cell`` as a mesh of
    their own (original relative order kept), with periodic images unwrapped
    around the centre cell.  Returns (patch mesh, patch cell ids)."""
    cells = inc.grow([centre_cell], rings)
    cn = mesh.cell_nodes[cells]
    nf = np.where(cn[:, 3] < 0, 3, 4)
    xy = mesh.node_xy
    # vertex averages (slot 3 of a triangle is -1 and ignored)
    cxy = np.stack([np.where(cn >= 0, xy[np.maximum(cn, 0), d], 0.0).sum(1) / nf
                    for d in (0, 1)], 1)
    centre = cxy[np.searchsorted(cells, centre_cell)]
    shift = np.zeros_like(cxy)
    for d in (0, 1):
        per = mesh.period[d]
        if per > 0:
            shift[:, d] = np.round((cxy[:, d] - centre[d]) / per) * -per
            # the patch must be small against the period for the images to be unique
            if np.abs(cxy[:, d] + shift[:, d] - centre[d]).max() >= 0.3 * per:
                raise PatchTooLarge(mesh.name)
    canon = inc.canon[cells]
    new_nodes = {}
    node_xy = []
    out = np.full(cn.shape, -1, dtype=np.int32)
    for r in range(cells.size):
        for k in range(nf[r]):
            p = (xy[cn[r, k], 0] + shift[r, 0], xy[cn[r, k], 1] + shift[r, 1])
            key = (int(canon[r, k]), p[0], p[1])
            j = new_nodes.get(key)
            if j is None:
                j = len(node_xy)
                new_nodes[key] = j
                node_xy.append(p)
            out[r, k] = j
    # real boundary faces keep their kind; the faces the cut opens take
    # whatever their row says, which cannot reach the centre cell
    fbc = getattr(mesh, "face_bc", None)
    sub = wl.Mesh(node_xy=np.array(node_xy, dtype=np.float64), cell_nodes=out, node_id=None,
                  period=(0.0, 0.0), bc="transmissive", h=mesh.h, name=f"patch{centre_cell}",
                  face_bc=None if fbc is None else np.asarray(fbc)[cells],
                  inflow=getattr(mesh, "inflow", None), fronts=getattr(mesh, "fronts", None))
    return sub, cells


def rk3_at(mesh, W, samples, physics, dt, steps=1, inc=None, scheme=None, t0=0.0):
    """Oracle state after ``steps`` RK3 steps of fixed ``dt`` from time t0 at
    the sampled cells (original ids): array [nvar, len(samples)]."""
    inc = inc or NodeIncidence(mesh)
    rings = RK3_RINGS * steps
    out = np.empty((W.shape[0], len(samples)))
    for s, c in enumerate(samples):
        try:
            sub, cells = patch_mesh(mesh, inc, int(c), rings)
        except PatchTooLarge:
            # a small periodic mesh: the whole-mesh oracle answers directly
            T = ow.precompute(mesh, scheme)
            Wt, t = W.copy(), t0
            for _ in range(steps):
                Wt = osc.rk3_step(T, Wt, physics, dt, t=t)
                t = t + dt
            return Wt[:, np.asarray(samples)]
        T = ow.precompute(sub, scheme)
        Ws = W[:, cells].copy()
        # cells at the patch edge see truncated stencils and may leave the
        # admissible set; they are out of the sampled cell's reach
        with np.errstate(invalid="ignore", divide="ignore"):
            t = t0
            for _ in range(steps):
                Ws = osc.rk3_step(T, Ws, physics, dt, t=t)
                t = t + dt   # the time is accumulated step by step
        out[:, s] = Ws[:, np.searchsorted(cells, c)]
    return out


def residual_at(mesh, W, samples, physics, inc=None, scheme=None, t=0.0):
    """Oracle residual L(W) at time t at the sampled cells (three rings suffice)."""
    inc = inc or NodeIncidence(mesh)
    out = np.empty((W.shape[0], len(samples)))
    for s, c in enumerate(samples):
        sub, cells = patch_mesh(mesh, inc, int(c), 3)
        T = ow.precompute(sub, scheme)
        L = osc.residual_vectorized(T, W[:, cells], physics, t=t)
        out[:, s] = L[:, np.searchsorted(cells, c)]
    return out
