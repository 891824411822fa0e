"""Seeded synthetic inputs: meshes, initial cell averages and exact solutions.

This module is shared by the oracle, the tests and the benchmark as the single
source of *inputs*.  It contains none of the scheme's arithmetic (no stencils,
no least squares, no weights, no fluxes): only node coordinates, cell-node
lists, and cell averages of closed-form fields, computed by a plain
high-order quadrature.

Meshes
------
All meshes are structured-derived: an ``nx`` by ``ny`` grid of squares of
side ``h`` whose interior nodes are moved by a seeded uniform jitter, each
square kept as one counter-clockwise quadrilateral or split into two
counter-clockwise triangles along its (i,j)-(i+1,j+1) diagonal; or
(``lattice_mesh``) rows of near-equilateral triangles.  The paper's
own test meshes (the "regular" and "irregular" families of its accuracy
section) exist only as figures; these jittered grids stand in for them.

* RNG: ``numpy.random.Generator(PCG64(seed))``; the jitter draws dx then dy,
  uniform in [-a h, a h], per interior node in row-major (j, i) order.
* Nodes on the domain boundary never move.  For periodic domains the seam
  nodes are duplicated, the duplicates offset by exactly the period, and
  ``node_id`` gives every node its canonical (wrapped) id.
* Inversion guard (a >= 0.25): up to five rounds; in each round every cell
  whose signed area is below 0.05 times its undeformed area halves the
  displacement of each of its nodes (the fifth time: sets it to zero).
  After the last round no cell is below the threshold.

The state layout everywhere is ``W[v, cell]`` (variables major), float64, in
the mesh's original cell order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GAMMA = 1.4


@dataclasses.dataclass
class Mesh:
    node_xy: np.ndarray          # float64 [n_nodes, 2]
    cell_nodes: np.ndarray       # int32 [n_cells, 4]; triangles have -1 in slot 3
    node_id: np.ndarray | None   # int32 [n_nodes] canonical ids (periodic), or None
    period: tuple                # (px, py); 0 = not periodic in that axis
    bc: str                      # "periodic" or "transmissive"
    h: float                     # nominal cell size
    name: str = ""
    # boundary kind of each unmatched face [n_cells, 4] (BC_* below; 0 = bc),
    # and the prescribed states that BC_INFLOW + s refers to [n_states, 4]
    face_bc: np.ndarray | None = None
    inflow: np.ndarray | None = None
    fronts: np.ndarray | None = None      # [n_fronts, 12] moving fronts (see BC_FRONT)

    @property
    def n_cells(self) -> int:
        return int(self.cell_nodes.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.node_xy.shape[0])

    def n_faces_of(self) -> np.ndarray:
        return np.where(self.cell_nodes[:, 3] < 0, 3, 4).astype(np.int32)


# boundary kinds of unmatched faces (input description only); a moving
# front f is BC_FRONT + f, its row in mesh.fronts = (ex, ey, c0, s, A, B)
BC_DEFAULT, BC_TRANSMISSIVE, BC_REFLECTIVE, BC_INFLOW, BC_FRONT = 0, 1, 2, 3, 1 << 16


# --------------------------------------------------------------------------
# mesh construction
# --------------------------------------------------------------------------

def _cells_from_split(nx: int, ny: int, split: np.ndarray) -> np.ndarray:
    """Cell-node list in row-major square order; a split square gives the
    triangles (i,j),(i+1,j),(i+1,j+1) then (i,j),(i+1,j+1),(i,j+1)."""
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    n00 = (jj * (nx + 1) + ii).ravel()
    n10 = n00 + 1
    n11 = n00 + nx + 2
    n01 = n00 + nx + 1
    sp = split.ravel()
    cnt = np.where(sp, 2, 1)
    start = np.cumsum(cnt) - cnt
    total = int(cnt.sum())
    cells = np.full((total, 4), -1, dtype=np.int32)
    q = ~sp
    cells[start[q]] = np.stack([n00[q], n10[q], n11[q], n01[q]], axis=1)
    s0 = start[sp]
    cells[s0, 0] = n00[sp]
    cells[s0, 1] = n10[sp]
    cells[s0, 2] = n11[sp]
    cells[s0 + 1, 0] = n00[sp]
    cells[s0 + 1, 1] = n11[sp]
    cells[s0 + 1, 2] = n01[sp]
    return cells


def signed_areas(node_xy: np.ndarray, cell_nodes: np.ndarray) -> np.ndarray:
    """Shoelace signed area of every cell (input validation / guard only)."""
    nf = np.where(cell_nodes[:, 3] < 0, 3, 4)
    x = node_xy[np.maximum(cell_nodes, 0), 0]
    y = node_xy[np.maximum(cell_nodes, 0), 1]
    a = np.zeros(cell_nodes.shape[0])
    for k in range(4):
        kn = np.where(k + 1 < nf, k + 1, 0)
        valid = k < nf
        xk = x[:, k]
        yk = y[:, k]
        xn = np.take_along_axis(x, kn[:, None], 1)[:, 0]
        yn = np.take_along_axis(y, kn[:, None], 1)[:, 0]
        a += np.where(valid, xk * yn - xn * yk, 0.0)
    return 0.5 * a


def grid_mesh(nx: int, ny: int, lx: float, ly: float, split, jitter: float,
              seed, periodic: bool, name: str = "") -> Mesh:
    """Jittered structured-derived mesh on [0,lx] x [0,ly].

    ``split`` is "quad", "tri" or a boolean array [ny, nx] (True = split the
    square into two triangles).  ``seed`` is an int or a SeedSequence.
    """
    h = lx / nx
    if isinstance(split, str):
        split = np.full((ny, nx), split == "tri")
    split = np.asarray(split, dtype=bool)
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    xs[-1] = lx
    ys[-1] = ly
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    node_xy = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    cells = _cells_from_split(nx, ny, split)

    rng = np.random.Generator(np.random.PCG64(seed))
    interior = np.zeros((ny + 1, nx + 1), dtype=bool)
    interior[1:-1, 1:-1] = True
    idx = np.flatnonzero(interior.ravel())
    disp = np.zeros_like(node_xy)
    if jitter > 0 and idx.size:
        disp[idx] = rng.uniform(-jitter * h, jitter * h, size=(idx.size, 2))
    base_area = np.where(cells[:, 3] < 0, 0.5 * h * h, h * h)
    xy = node_xy + disp
    if jitter >= 0.25:
        halvings = np.zeros(node_xy.shape[0], dtype=np.int32)
        for _ in range(5):
            a = signed_areas(xy, cells)
            bad = a < 0.05 * base_area
            if not bad.any():
                break
            nodes = np.unique(cells[bad][cells[bad] >= 0])
            halvings[nodes] += 1
            disp[nodes] *= 0.5
            disp[nodes[halvings[nodes] >= 5]] = 0.0
            xy = node_xy + disp
    node_xy = xy
    a = signed_areas(node_xy, cells)
    if not (a > 0).all():
        raise RuntimeError("mesh generator produced a non-positive cell area")
    node_id = None
    period = (0.0, 0.0)
    if periodic:
        jj, ii = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
        node_id = ((jj % ny) * nx + (ii % nx)).ravel().astype(np.int32)
        period = (float(lx), float(ly))
    return Mesh(node_xy=node_xy, cell_nodes=cells, node_id=node_id, period=period,
                bc="periodic" if periodic else "transmissive", h=h, name=name)


# --------------------------------------------------------------------------
# the five workloads (plus refinements used for convergence studies)
# --------------------------------------------------------------------------

def mesh_c1(n: int = 20, jitter: float = 0.10, seed=1) -> Mesh:
    """Scalar advection mesh: n x n squares on [0,2]^2, all split, periodic."""
    return grid_mesh(n, n, 2.0, 2.0, "tri", jitter, seed, True, name=f"tri{n}")


def mesh_c2q(n: int = 400, jitter: float = 0.20, seed=2) -> Mesh:
    return grid_mesh(n, n, 2.0, 2.0, "quad", jitter, seed, True, name=f"quad{n}")


def mesh_c2t(n: int = 283, jitter: float = 0.20, seed=3) -> Mesh:
    return grid_mesh(n, n, 2.0, 2.0, "tri", jitter, seed, True, name=f"tri{n}")


def mesh_c3(n: int = 1340, jitter: float = 0.15, seed=4, band: float = 0.05) -> Mesh:
    """Rotated shock tube on [0,1]^2: squares whose centre lies within ``band``
    of the interface line are split; transmissive boundaries."""
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    cx, cy = np.meshgrid(c, c, indexing="xy")
    nx_, ny_ = math.cos(math.pi / 6), math.sin(math.pi / 6)
    dist = np.abs((cx - 0.5) * nx_ + (cy - 0.5) * ny_)
    return grid_mesh(n, n, 1.0, 1.0, dist < band, jitter, seed, False, name=f"sod{n}")


def mesh_c5(n: int = 3264, block: int = 64, jitter: float = 0.30, seed=6) -> Mesh:
    """Large mixed periodic mesh on [0,2]^2: n x n squares in block x block
    tiles, checkerboard; tiles with (bi + bj) odd are split into triangles."""
    b = np.arange(n) // block
    bj, bi = np.meshgrid(b, b, indexing="ij")
    split = ((bi + bj) % 2) == 1
    return grid_mesh(n, n, 2.0, 2.0, split, jitter, seed, True, name=f"mixed{n}")


def c4_instances(count: int = 256, seed: int = 5, nmin: float = 2e3, nmax: float = 2e5):
    """Parameters of the batched workload: per instance (kind, n, jitter, seed).

    N_k is log-uniform in [nmin, nmax]; the mesh type is a fair coin; the
    jitter amplitude is uniform in [0, 0.3]; the mesh seed is the k-th child
    of SeedSequence(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    logn = rng.uniform(math.log(nmin), math.log(nmax), size=count)
    is_tri = rng.random(count) < 0.5
    amp = rng.uniform(0.0, 0.3, size=count)
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for k in range(count):
        nk = math.exp(logn[k])
        if is_tri[k]:
            n = max(4, int(round(math.sqrt(nk / 2))))
        else:
            n = max(4, int(round(math.sqrt(nk))))
        out.append(("tri" if is_tri[k] else "quad", n, float(amp[k]), children[k]))
    return out


def mesh_c4(k: int, count: int = 256) -> Mesh:
    kind, n, amp, ss = c4_instances(count)[k]
    return grid_mesh(n, n, 2.0, 2.0, kind, amp, ss, True, name=f"batch{k}")


# --------------------------------------------------------------------------
# cell averages by quadrature (input preparation only)
# --------------------------------------------------------------------------

def _triangle_rule(q: int):
    """Collapsed (Duffy) Gauss-Legendre rule on the reference triangle
    {(s,t): s,t >= 0, s + t <= 1}; exact for total degree 2q - 2."""
    g, w = np.polynomial.legendre.leggauss(q)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    U, V = np.meshgrid(g, g, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    s = U.ravel()
    t = (V * (1.0 - U)).ravel()
    wt = (WU * WV * (1.0 - U)).ravel()
    return s, t, wt  # weights sum to 1/2


def cell_averages(mesh: Mesh, fn, nvar: int, q: int = 4, chunk: int = 1 << 18) -> np.ndarray:
    """Average of ``fn(x, y) -> [nvar, ...]`` over every cell, integrating a
    fan of triangles from vertex 0 with a collapsed Gauss rule."""
    s, t, wt = _triangle_rule(q)
    out = np.empty((nvar, mesh.n_cells))
    cn = mesh.cell_nodes
    for c0 in range(0, mesh.n_cells, chunk):
        c1 = min(mesh.n_cells, c0 + chunk)
        nodes = cn[c0:c1]
        nf = np.where(nodes[:, 3] < 0, 3, 4)
        p = mesh.node_xy[np.maximum(nodes, 0)]  # [m, 4, 2]
        acc = np.zeros((nvar, c1 - c0))
        area = np.zeros(c1 - c0)
        for k in (1, 2):
            valid = np.ones(c1 - c0, dtype=bool) if k == 1 else (nf == 4)
            a = p[:, 0]
            b = p[:, k]
            c = p[:, k + 1]
            e1 = b - a
            e2 = c - a
            jac = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
            x = a[:, None, 0] + e1[:, None, 0] * s[None] + e2[:, None, 0] * t[None]
            y = a[:, None, 1] + e1[:, None, 1] * s[None] + e2[:, None, 1] * t[None]
            f = np.asarray(fn(x, y))  # [nvar, m, nq]
            contrib = (f * wt[None, None, :]).sum(axis=-1) * jac[None, :]
            acc += np.where(valid[None, :], contrib, 0.0)
            area += np.where(valid, 0.5 * jac, 0.0)
        out[:, c0:c1] = acc / area[None, :]
    return out


# --------------------------------------------------------------------------
# closed-form fields
# --------------------------------------------------------------------------

def density_wave_scalar(t: float = 0.0, a=(1.0, 1.0)):
    def f(x, y):
        return (1.0 + 0.2 * np.sin(np.pi * ((x - a[0] * t) + (y - a[1] * t))))[None]
    return f


def primitive_to_conserved(rho, u, v, p, gamma=GAMMA):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def density_wave_euler(t: float = 0.0, gamma=GAMMA):
    """rho = 1 + 0.2 sin(pi(x + y - 2t)), u = v = p = 1 (exact for all t)."""
    def f(x, y):
        rho = 1.0 + 0.2 * np.sin(np.pi * (x + y - 2.0 * t))
        one = np.ones_like(rho)
        return primitive_to_conserved(rho, one, one, one, gamma)
    return f


def wave_vortex_euler(strength: float = 5.0, centre=(1.0, 1.0), scale: float = 5.0,
                      gamma=GAMMA):
    """Density wave times an isentropic vortex evaluated at
    (xb, yb) = scale * (x - xc, y - yc) (initial data of the large mixed mesh)."""
    def f(x, y):
        xb = scale * (x - centre[0])
        yb = scale * (y - centre[1])
        r2 = xb * xb + yb * yb
        du = strength / (2 * np.pi) * np.exp(0.5 * (1 - r2)) * (-yb)
        dv = strength / (2 * np.pi) * np.exp(0.5 * (1 - r2)) * xb
        dT = -(gamma - 1) * strength ** 2 / (8 * gamma * np.pi ** 2) * np.exp(1 - r2)
        rho = (1.0 + 0.2 * np.sin(np.pi * (x + y))) * (1 + dT) ** (1 / (gamma - 1))
        p = (1 + dT) ** (gamma / (gamma - 1))
        return primitive_to_conserved(rho, 1.0 + du, 1.0 + dv, p, gamma)
    return f


def isentropic_vortex(t: float = 0.0, strength: float = 5.0, centre=(5.0, 5.0),
                      period: float = 10.0, gamma=GAMMA):
    """The paper's isentropic vortex (Sec. 4.1): mean flow (1, 1, 1, 1) plus
    (du, dv) = s/(2 pi) e^{(1 - r^2)/2} (-yb, xb), dT = -(gamma - 1) s^2
    / (8 gamma pi^2) e^{1 - r^2}, isentropic, advected by the mean flow to
    time t on a periodic square of side ``period`` (nearest image)."""
    def f(x, y):
        xb = (x - centre[0] - t + period / 2) % period - period / 2
        yb = (y - centre[1] - t + period / 2) % period - period / 2
        r2 = xb * xb + yb * yb
        du = strength / (2 * np.pi) * np.exp(0.5 * (1 - r2)) * (-yb)
        dv = strength / (2 * np.pi) * np.exp(0.5 * (1 - r2)) * xb
        dT = -(gamma - 1) * strength ** 2 / (8 * gamma * np.pi ** 2) * np.exp(1 - r2)
        rho = (1 + dT) ** (1 / (gamma - 1))
        p = (1 + dT) ** (gamma / (gamma - 1))
        return primitive_to_conserved(rho, 1.0 + du, 1.0 + dv, p, gamma)
    return f


def rotated_sod(angle_deg: float = 30.0, gamma=GAMMA):
    """Sod states (1,0,0,1) | (0.125,0,0,0.1) across the line through
    (0.5,0.5) with unit normal (cos a, sin a); left where (x-0.5,y-0.5).n < 0."""
    ca, sa = math.cos(math.radians(angle_deg)), math.sin(math.radians(angle_deg))

    def f(x, y):
        left = ((x - 0.5) * ca + (y - 0.5) * sa) < 0
        rho = np.where(left, 1.0, 0.125)
        p = np.where(left, 1.0, 0.1)
        z = np.zeros_like(rho)
        return primitive_to_conserved(rho, z, z, p, gamma)
    return f


def sod_cell_values(mesh: Mesh, angle_deg: float = 30.0, gamma=GAMMA) -> np.ndarray:
    """Sod initial data sampled at vertex averages (a discontinuous field has
    no useful quadrature; the cell takes the state at its vertex average)."""
    cn = mesh.cell_nodes
    nf = np.where(cn[:, 3] < 0, 3, 4)
    p = mesh.node_xy[np.maximum(cn, 0)]
    cx = (p[:, 0, 0] + p[:, 1, 0] + p[:, 2, 0] + np.where(nf == 4, p[:, 3, 0], 0.0)) / nf
    cy = (p[:, 0, 1] + p[:, 1, 1] + p[:, 2, 1] + np.where(nf == 4, p[:, 3, 1], 0.0)) / nf
    return rotated_sod(angle_deg, gamma)(cx, cy)


def seeded_state(mesh: Mesh, nvar: int, seed: int, amp: float = 0.1) -> np.ndarray:
    """A smooth field plus seeded cell noise: a generic non-trivial state for
    parity tests (positive density and pressure for the Euler case)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if nvar == 1:
        base = cell_averages(mesh, density_wave_scalar(0.0), 1, q=3)
    else:
        base = cell_averages(mesh, density_wave_euler(0.0), 4, q=3)
    noise = rng.uniform(-amp, amp, size=base.shape)
    if nvar == 4:
        noise[1:3] *= 1.0
        noise[3] *= 2.0
    return base + noise


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

WORKLOADS = {
    "c1": dict(equation="advection", t_end=0.2, cfl=0.5, nvar=1),
    "c2q": dict(equation="euler", t_end=0.5, cfl=0.5, nvar=4),
    "c2t": dict(equation="euler", t_end=0.5, cfl=0.5, nvar=4),
    "c3": dict(equation="euler", t_end=0.2, cfl=0.5, nvar=4),
    "c4": dict(equation="euler", steps=100, cfl=0.5, nvar=4),
    "c5": dict(equation="euler", steps=50, cfl=0.5, nvar=4),
}


# --------------------------------------------------------------------------
# boundary kinds and the paper's other test problems (Sec. 4.2-4.4)
# --------------------------------------------------------------------------

def set_face_kinds(mesh: Mesh, kind_of) -> Mesh:
    """Fill mesh.face_bc from ``kind_of(mx, my, nx, ny)`` evaluated at every
    face's midpoint with its outward normal (the library and the oracle read
    it only on unmatched faces)."""
    cn = mesh.cell_nodes
    nf = np.where(cn[:, 3] < 0, 3, 4)
    kinds = np.zeros((mesh.n_cells, 4), np.int32)
    for k in range(4):
        valid = k < nf
        a = mesh.node_xy[np.maximum(cn[:, k], 0)]
        nxt = np.where(k + 1 < nf, (k + 1) % 4, 0)
        b = mesh.node_xy[np.maximum(cn[np.arange(mesh.n_cells), nxt], 0)]
        m = 0.5 * (a + b)
        t = b - a
        ln = np.maximum(np.hypot(t[:, 0], t[:, 1]), 1e-300)
        kinds[:, k] = np.where(valid, kind_of(m[:, 0], m[:, 1], t[:, 1] / ln, -t[:, 0] / ln), 0)
    mesh.face_bc = kinds
    return mesh


def box_mesh(kind: int, n: int = 12, jitter: float = 0.25, seed: int = 3,
             inflow=None) -> Mesh:
    """Open unit square, n x n squares in 3 x 3 blocks alternating between
    quadrilaterals and split triangles, every boundary face of one kind."""
    split = (np.add.outer(np.arange(n) // 3, np.arange(n) // 3) % 2).astype(bool)
    mesh = grid_mesh(n, n, 1.0, 1.0, split, jitter, seed, False, name=f"box{kind}-{n}")
    mesh.face_bc = np.full((mesh.n_cells, 4), kind, dtype=np.int32)
    if inflow is not None:
        mesh.inflow = np.asarray(inflow, dtype=np.float64).reshape(-1, 4)
    return mesh


def channel_mesh(nx: int = 20, ny: int = 10, split="tri", jitter: float = 0.2, seed: int = 9,
                 inflow=None, lx: float = 2.0, ly: float = 1.0) -> Mesh:
    """Channel [0,lx] x [0,ly]: slip walls top and bottom, the prescribed
    state 0 entering on the left, an open right end."""
    mesh = grid_mesh(nx, ny, lx, ly, split, jitter, seed, False, name=f"channel{nx}x{ny}")
    tol = 1e-9 * max(lx, ly)

    def kind_of(mx, my, nx_, ny_):
        wall = (np.abs(my) < tol) | (np.abs(my - ly) < tol)
        left = np.abs(mx) < tol
        return np.where(wall, BC_REFLECTIVE, np.where(left, BC_INFLOW, BC_TRANSMISSIVE))
    set_face_kinds(mesh, kind_of)
    if inflow is not None:
        mesh.inflow = np.asarray(inflow, dtype=np.float64).reshape(-1, 4)
    return mesh


def lax_state(mesh: Mesh, gamma=GAMMA) -> np.ndarray:
    """Lax problem (Sec. 4.2): (0.445, 0.698, 3.528) for x < 0.5, else
    (0.5, 0, 0.571), sampled at vertex averages."""
    cx, cy = cell_centres(mesh)
    left = cx < 0.5
    rho = np.where(left, 0.445, 0.5)
    u = np.where(left, 0.698, 0.0)
    p = np.where(left, 3.528, 0.571)
    return primitive_to_conserved(rho, u, np.zeros_like(u), p, gamma)


RIEMANN_1D = {   # (rho, u, p) left and right, end time (Sec. 4.2)
    "sod": ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.2),
    "lax": ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571), 0.16),
}


def riemann_1d(problem: str = "sod", n: int = 100, split="quad", jitter: float = 0.0,
               seed: int = 7, gamma=GAMMA):
    """One-dimensional Riemann problem as the paper sets it (Sec. 4.2): the
    states of RIEMANN_1D split at x = 0.5 on [0,1] x [0,0.5], h = 1/n, open
    (transmissive) boundaries.  ``split``: "quad", "tri" (split squares,
    jittered by ``jitter``) or "lattice" (near-equilateral triangles).
    Returns (mesh, state, end time); cells take the state at their vertex
    average."""
    left, right, t_end = RIEMANN_1D[problem]
    if split == "lattice":
        mesh = lattice_mesh(n, int(round(0.5 * n / (math.sqrt(3.0) / 2))), 1.0, 0.5,
                            name=f"{problem}-lattice{n}")
    else:
        mesh = grid_mesh(n, n // 2, 1.0, 0.5, split, jitter, seed, False,
                         name=f"{problem}-{split}{n}")
    cx, _ = cell_centres(mesh)
    lft = cx < 0.5
    W = primitive_to_conserved(np.where(lft, left[0], right[0]), np.where(lft, left[1], right[1]),
                               np.zeros_like(cx), np.where(lft, left[2], right[2]), gamma)
    return mesh, W, t_end


def shu_osher(nx: int = 400, ny: int = 10, jitter: float = 0.3, seed: int = 11,
              split="quad", gamma=GAMMA):
    """Shu-Osher problem as the paper sets it (Sec. 4.2): [0,10] x [0,0.25],
    (3.857134, 2.629369, 10.33333) for x <= 1, else (1 + 0.2 sin 5x, 0, 1);
    slip walls in y, the left state entering on the left, open right end.
    Returns (mesh, state)."""
    left = primitive_to_conserved(3.857134, 2.629369, 0.0, 10.33333, gamma)
    mesh = channel_mesh(nx, ny, split, jitter, seed, inflow=np.asarray(left), lx=10.0, ly=0.25)

    def f(x, y):
        rho = np.where(x <= 1.0, 3.857134, 1.0 + 0.2 * np.sin(5.0 * x))
        u = np.where(x <= 1.0, 2.629369, 0.0)
        p = np.where(x <= 1.0, 10.33333, 1.0)
        return primitive_to_conserved(rho, u, np.zeros_like(u), p, gamma)
    return mesh, cell_averages(mesh, f, 4, q=3)


def shock_vortex(n: int = 100, jitter: float = 0.3, seed: int = 12, split="tri",
                 gamma=GAMMA, mach: float = 1.1, kappa: float = 0.3, mu: float = 0.204,
                 rc: float = 0.05, centre=(0.25, 0.5)):
    """Shock-vortex interaction (Sec. 4.3): [0,2] x [0,1], a stationary
    Mach 1.1 shock at x = 0.5 with upstream (rho, U, V, p) = (Ma^2, sqrt(gamma),
    0, 1), the downstream state from the Rankine-Hugoniot relations, and the
    vortex perturbation of the paper added upstream; slip walls top and
    bottom, the upstream state entering on the left, open right end.
    Returns (mesh, state)."""
    r1, u1, p1 = mach ** 2, math.sqrt(gamma), 1.0
    m2 = mach ** 2
    r2 = r1 * (gamma + 1) * m2 / ((gamma - 1) * m2 + 2)
    p2 = p1 * (2 * gamma * m2 - (gamma - 1)) / (gamma + 1)
    u2 = r1 * u1 / r2
    up = np.asarray(primitive_to_conserved(r1, u1, 0.0, p1, gamma))
    mesh = channel_mesh(2 * n, n, split, jitter, seed, inflow=up, lx=2.0, ly=1.0)

    def f(x, y):
        dx, dy = x - centre[0], y - centre[1]
        eta = np.hypot(dx, dy) / rc
        th = np.arctan2(dy, dx)
        amp = kappa * eta * np.exp(mu * (1 - eta * eta))
        du, dv = amp * np.sin(th), -amp * np.cos(th)
        dT = -(gamma - 1) * kappa ** 2 / (4 * mu * gamma) * np.exp(2 * mu * (1 - eta * eta))
        # upstream: T = p / rho and S = ln(p / rho^gamma) fixed, T perturbed
        T = p1 / r1 + dT
        rho_v = (T / (p1 / r1 ** gamma)) ** (1.0 / (gamma - 1))
        up_ = x < 0.5
        rho = np.where(up_, rho_v, r2)
        u = np.where(up_, u1 + du, u2)
        v = np.where(up_, dv, 0.0)
        p = np.where(up_, rho_v * T, p2)
        return primitive_to_conserved(rho, u, v, p, gamma)
    return mesh, cell_averages(mesh, f, 4, q=3)


def lattice_mesh(nx: int, ny: int, lx: float, ly: float, name: str = "") -> Mesh:
    """Near-equilateral triangles on [0,lx] x [0,ly]: ny + 1 rows of nodes,
    odd rows shifted by half the spacing lx/nx (their end nodes kept on
    x = 0 and x = lx), each strip between two rows zipped into triangles
    from left to right.  With ny = ly/(lx/nx)/(sqrt3/2) the interior
    triangles are equilateral."""
    hx = lx / nx
    rows, xy = [], []
    for j in range(ny + 1):
        y = ly * j / ny
        xs = ([i * hx for i in range(nx + 1)] if j % 2 == 0
              else [0.0] + [(i + 0.5) * hx for i in range(nx)] + [lx])
        rows.append(list(range(len(xy), len(xy) + len(xs))))
        xy += [(x, y) for x in xs]
    xy = np.array(xy, dtype=np.float64)
    cells = []
    for j in range(ny):
        b, top = rows[j], rows[j + 1]
        ib = it = 0
        while ib < len(b) - 1 or it < len(top) - 1:
            if it == len(top) - 1 or (ib < len(b) - 1 and xy[b[ib + 1], 0] <= xy[top[it + 1], 0]):
                cells.append((b[ib], b[ib + 1], top[it], -1))
                ib += 1
            else:
                cells.append((b[ib], top[it + 1], top[it], -1))
                it += 1
    return Mesh(node_xy=xy, cell_nodes=np.array(cells, dtype=np.int32), node_id=None,
                period=(0.0, 0.0), bc="transmissive", h=hx, name=name or f"lattice{nx}x{ny}")


def double_mach(nx: int = 400, ny: int = 100, split="tri", jitter: float = 0.15, seed: int = 13,
                gamma=GAMMA, t: float = 0.0):
    """Double Mach reflection (Sec. 4.4): [0,4] x [0,1], a Mach 10 shock
    through (1/6, 0) at 60 degrees to the x-axis, post-shock state
    (8, 4.125 sqrt3, -4.125, 116.5) behind it and (1.4, 0, 0, 1) ahead.  The
    bottom is a slip wall from x = 1/6 on and carries the post-shock state
    before it, the left end takes the post-shock state, the right end is
    open, and the top follows the exact shock: post-shock where
    x < 1/6 + (1 + 20 t)/sqrt3, else pre-shock.  The state is the incident
    shock alone at time t (the exact solution at t = 0; later, away from the
    reflection that forms at the wall).  split "quad" or "tri" (squares,
    split along a diagonal, jittered) or "lattice" (near-equilateral
    triangles of side 4/nx, ny ignored).  Returns (mesh, state)."""
    post = np.asarray(primitive_to_conserved(8.0, 4.125 * math.sqrt(3.0), -4.125, 116.5, gamma))
    pre = np.asarray(primitive_to_conserved(1.4, 0.0, 0.0, 1.0, gamma))
    if split == "lattice":
        rows = int(round(nx / 4.0 / (math.sqrt(3.0) / 2.0)))
        mesh = lattice_mesh(nx, rows, 4.0, 1.0, name=f"dmr-lattice{nx}x{rows}")
    else:
        mesh = grid_mesh(nx, ny, 4.0, 1.0, split, jitter, seed, False, name=f"dmr{nx}x{ny}")
    x0, r3 = 1.0 / 6.0, math.sqrt(3.0)
    tol = 1e-9

    def kind_of(mx, my, nx_, ny_):
        bottom = np.abs(my) < tol
        top = np.abs(my - 1.0) < tol
        left = np.abs(mx) < tol
        k = np.full(mx.shape, BC_TRANSMISSIVE)
        k = np.where(left, BC_INFLOW, k)
        k = np.where(bottom, np.where(mx < x0, BC_INFLOW, BC_REFLECTIVE), k)
        return np.where(top, BC_FRONT, k)
    set_face_kinds(mesh, kind_of)
    mesh.inflow = post[None, :].copy()
    mesh.fronts = np.concatenate([[1.0, 0.0, x0 + 1.0 / r3, 20.0 / r3], post, pre])[None, :]
    cx, cy = cell_centres(mesh)
    behind = cx < x0 + (cy + 20.0 * t) / r3
    W = np.where(behind[None, :], post[:, None], pre[:, None])
    return mesh, W


def cell_centres(mesh: Mesh):
    """Vertex averages of the cells (x, y)."""
    cn = mesh.cell_nodes
    nf = np.where(cn[:, 3] < 0, 3, 4)
    xy = np.where((cn >= 0)[:, :, None], mesh.node_xy[np.maximum(cn, 0)], 0.0).sum(1)
    return xy[:, 0] / nf, xy[:, 1] / nf


def initial_state(name: str, mesh: Mesh, q: int | None = None) -> np.ndarray:
    if name == "c1":
        return cell_averages(mesh, density_wave_scalar(0.0), 1, q=q or 5)
    if name in ("c2q", "c2t", "c4"):
        return cell_averages(mesh, density_wave_euler(0.0), 4, q=q or 4)
    if name == "c3":
        return sod_cell_values(mesh)
    if name == "c5":
        return cell_averages(mesh, wave_vortex_euler(), 4, q=q or 2)
    raise KeyError(name)
