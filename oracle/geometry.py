"""Oracle: cell geometry in the scaled frame of each target cell.

Test infrastructure only (see the package docstring).

Paper: Sec. 2 (face length |l_p|, outer normal n_p, the two Gauss points of
eq. (quadrature): x_p1 = (3+sqrt3)/6 X_p1 + (3-sqrt3)/6 X_p2 and the mirror
x_p2), Sec. 3.1 (zero-mean quadratic basis of eq. (base); cell averages of
the basis functions in the constraint matrix A).

Reading: all polynomials of a target cell i0 are written in the scaled local
coordinates xi = (x - xbar_i0) / h0 with h0 = sqrt(|Omega_i0|); the basis
p^k - <p^k>_{i0} spans the same space as eq. (base), and the regularisation
parameter zeta of eq. (quadratic-2) then acts on dimensionless quantities.
Polygon moments up to degree two are integrated exactly: a signed fan of
triangles from vertex 0, each integrated with the edge-midpoint rule.
"""
from __future__ import annotations

import math

import numpy as np

GP_A = (3.0 + math.sqrt(3.0)) / 6.0
GP_B = (3.0 - math.sqrt(3.0)) / 6.0


def cell_polygons(mesh, ids):
    """Vertices [m,4,2] (slot 3 repeats vertex 0 for triangles) and face count."""
    cn = np.asarray(mesh.cell_nodes, dtype=np.int64)[ids]
    nf = np.where(cn[:, 3] < 0, 3, 4)
    P = np.asarray(mesh.node_xy, dtype=np.float64)[np.maximum(cn, 0)]
    P[:, 3] = np.where((nf == 4)[:, None], P[:, 3], P[:, 0])
    return P, nf


def poly_moments(P, nf):
    """Exact integrals of 1, x, y, x^2, y^2, xy over polygons P[...,4,2]
    (counter-clockwise), by a signed triangle fan from vertex 0 and the
    three-edge-midpoint rule on each triangle."""
    out = np.zeros(P.shape[:-2] + (6,))
    for k in (1, 2):
        use = (nf == 4) if k == 2 else np.ones_like(nf, dtype=bool)
        p0, p1, p2 = P[..., 0, :], P[..., k, :], P[..., k + 1, :]
        t = 0.5 * ((p1[..., 0] - p0[..., 0]) * (p2[..., 1] - p0[..., 1])
                   - (p2[..., 0] - p0[..., 0]) * (p1[..., 1] - p0[..., 1]))
        mids = (0.5 * (p0 + p1), 0.5 * (p1 + p2), 0.5 * (p2 + p0))
        f = np.zeros(P.shape[:-2] + (6,))
        for m in mids:
            x, y = m[..., 0], m[..., 1]
            f += np.stack([np.ones_like(x), x, y, x * x, y * y, x * y], axis=-1)
        out += np.where(use[..., None], (t / 3.0)[..., None] * f, 0.0)
    return out


def reflect(P, a, b):
    """Mirror points P[...,2] across the line through a and b."""
    d = b - a
    nrm = np.stack([d[..., 1], -d[..., 0]], axis=-1)
    nrm = nrm / np.linalg.norm(nrm, axis=-1, keepdims=True)
    s = ((P - a[..., None, :]) * nrm[..., None, :]).sum(-1)
    return P - 2.0 * s[..., None] * nrm[..., None, :]


class Frame:
    """Scaled frame of a group of target cells: centroid, h0, area, and the
    cell averages of the zero-mean basis over every present stencil slot."""

    def __init__(self, mesh, st):
        P0, nf0 = cell_polygons(mesh, st.cells)
        self.nf = nf0
        # centroid and area from moments relative to vertex 0 (raw units)
        rel = P0 - P0[:, :1, :]
        mom = poly_moments(rel, nf0)
        self.area = mom[:, 0]
        self.centroid = P0[:, 0, :] + mom[:, 1:3] / mom[:, 0:1]
        self.h0 = np.sqrt(self.area)
        self.raw_polygon = P0
        self.xi_polygon = self.to_xi(P0)
        # slot polygons in the target's xi frame
        m, S = st.cell.shape
        Pslot = np.zeros((m, S, 4, 2))
        nfs = np.full((m, S), 3)
        for j in range(S):
            real = st.present[:, j] & (st.ghost[:, j] < 0)
            ids = np.where(real, st.cell[:, j], st.cells)
            Pj, nfj = cell_polygons(mesh, ids)
            Pj = Pj + st.shift[:, j][:, None, :]
            Xj = self.to_xi(Pj)
            g = st.ghost[:, j]
            if (g >= 0).any():
                k = np.maximum(g, 0)
                a = self.xi_polygon[np.arange(m), k]
                b = self.xi_polygon[np.arange(m), (k + 1) % nf0]
                R = reflect(self.xi_polygon, a, b)
                # reflection reverses orientation: re-order to counter-clockwise
                Rq = R[:, [0, 3, 2, 1]]
                Rt = R[:, [0, 2, 1, 0]]
                Rr = np.where((nf0 == 4)[:, None, None], Rq, Rt)
                Xj = np.where((g >= 0)[:, None, None], Rr, Xj)
                nfj = np.where(g >= 0, nf0, nfj)
            Pslot[:, j] = Xj
            nfs[:, j] = nfj
        mo = poly_moments(Pslot, nfs)
        self.slot_area = mo[..., 0]
        avg = mo[..., 1:] / mo[..., :1]          # <xi>, <eta>, <xi^2>, <eta^2>, <xi eta>
        self.mean0 = avg[:, 0, :].copy()          # means over the target itself
        # cell averages of the zero-mean basis functions over each slot
        self.basis_avg = avg - self.mean0[:, None, :]
        self.present = st.present

    def to_xi(self, P):
        return (P - self.centroid[:, None, :]) / self.h0[:, None, None]

    def basis_at(self, xi):
        """Zero-mean basis p^1..p^5 at points xi[...,2] (same batch as the frame)."""
        x, y = xi[..., 0], xi[..., 1]
        m0 = self.mean0.reshape(self.mean0.shape[:1] + (1,) * (xi.ndim - 2) + (5,))
        return np.stack([x, y, x * x, y * y, x * y], axis=-1) - m0


def face_geometry(frame):
    """Per target cell and face k: length |l_k|, unit outer normal, and the two
    Gauss points in the xi frame (ordered from v_k towards v_{k+1})."""
    P = frame.raw_polygon
    nf = frame.nf
    m = P.shape[0]
    length = np.zeros((m, 4))
    normal = np.zeros((m, 4, 2))
    gp_xi = np.zeros((m, 4, 2, 2))
    for k in range(4):
        valid = k < nf
        kn = np.where(k + 1 < nf, k + 1, 0)
        a = P[:, k]
        b = P[np.arange(m), kn]
        e = b - a
        ln = np.where(valid, np.sqrt(e[:, 0] ** 2 + e[:, 1] ** 2), 1.0)
        length[:, k] = np.where(valid, ln, 0.0)
        normal[:, k, 0] = np.where(valid, e[:, 1] / ln, 0.0)
        normal[:, k, 1] = np.where(valid, -e[:, 0] / ln, 0.0)
        g1 = GP_A * a + GP_B * b
        g2 = GP_B * a + GP_A * b
        gp_xi[:, k, 0] = frame.to_xi(g1[:, None, :])[:, 0]
        gp_xi[:, k, 1] = frame.to_xi(g2[:, None, :])[:, 0]
    return length, normal, gp_xi
