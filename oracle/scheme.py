"""Oracle: WENO point values, numerical flux, residual, SSP-RK3, time step.

Test infrastructure only (see the package docstring).

Paper:
* Sec. 3.4: split of the optimised linear weights (theta = 3),
  gamma~+ = (gamma + theta|gamma|)/2, gamma~- = gamma~+ - gamma,
  sigma^pm = sum gamma~pm, gamma^pm = gamma~pm / sigma^pm; the new smoothness
  indicator beta~ = beta (1 + gamma^pm beta + (gamma^pm beta)^2) with
  beta_j = |Omega| int |grad P_j|^2 for the linear candidates; nonlinear
  weights alpha = gamma^pm / (beta~ + eps)^2, delta = alpha / sum alpha; the
  split reconstruction R = sigma^+ R^+ - sigma^- R^-.
* Sec. 2: eq. (semidiscrete) residual, eq. (quadrature) two-point Gauss rule
  with weights 1/2, eq. (transform) rotation to the face frame, HLLC flux.
* Sec. 4: the three-stage TVD Runge-Kutta scheme.

* Sec. 4 (Euler systems): the reconstruction may be carried out on the
  characteristic variables U = R^-1 W of Roe's mean matrix
  n_x dF/dW + n_y dG/dW at the quadrature point, the reconstructed values
  being projected back with R.

Readings:
* characteristic variables: the Roe mean is taken between the two cells
  that share the face of the quadrature point (cell averages; a boundary
  face uses the cell itself), with that face's outward normal; both points
  of a face share the projection.  The candidate polynomials, their
  smoothness indicators and the point values are all projected, and the
  nonlinear weights are formed per characteristic field;
* the final reconstruction keeps the factors sigma^pm of the split form and
  is evaluated about W_i0: R = W_i0 + sigma^+ sum delta^+ (P_j - W_i0)
  - sigma^- sum delta^- (P_j - W_i0) (equal to the split form because
  sum delta^pm = 1 and sigma^+ - sigma^- = sum gamma = 1);
* eps = 1e-3 (the paper leaves it unspecified; with 1e-6 the smooth
  advection test does not reach third order on meshes of the paper's sizes);
* HLLC: Toro's contact-restoring solver with the Davis wave-speed estimates
  S_L = min(u_L - a_L, u_R - a_R), S_R = max(u_L + a_L, u_R + a_R);
* every face flux is evaluated in a canonical orientation: the left state is
  the cell with the lower original id, the normal is that cell's outer
  normal, and both cells use the same value with opposite signs;
* boundary faces (the paper names the conditions of its tests but does not
  define them): the state outside a face is the inner reconstructed state
  (transmissive, "non-reflecting"), the inner state with its normal
  momentum reversed (reflective, a slip wall), or a prescribed state
  (inflow).  The same outside state, formed from the cell average, is the
  value of the mirrored ghost cell in the face neighbour's stencil slot;
  for scalar advection a wall is treated as transmissive.  A moving front
  (for the exact shock of the double Mach reflection) gives one of two
  prescribed states by the side of a moving line on which the face
  midpoint lies, at the time of the RK stage (t, t + dt, t + dt/2);
* time step: dt = CFL min_i 2|Omega_i| / sum_p |l_p| (|u_i . n_p| + c_i), from
  cell averages (c = 0 and u = a for scalar advection), clamped to t_end - t.
  The paper instead fixes dt = 0.3 h for its accuracy runs.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .weights import Tables, group_row  # noqa: F401


@dataclasses.dataclass
class Physics:
    equation: str = "euler"     # "euler" or "advection"
    ax: float = 1.0
    ay: float = 1.0
    gamma: float = 1.4

    @property
    def nvar(self) -> int:
        return 4 if self.equation == "euler" else 1


# --------------------------------------------------------------------------
# boundary faces
# --------------------------------------------------------------------------

BC_TRANSMISSIVE, BC_REFLECTIVE, BC_INFLOW, BC_FRONT = 1, 2, 3, 1 << 16


def face_kind(mesh, cells, k):
    """Boundary kind of face k of the given cells (meaningful where the face
    is unmatched): the per-face kind, else the mesh's default."""
    cells = np.asarray(cells)
    kind = np.full(cells.shape, BC_TRANSMISSIVE, dtype=np.int64)
    if getattr(mesh, "face_bc", None) is not None:
        fk = np.asarray(mesh.face_bc)[cells, k].astype(np.int64)
        kind = np.where(fk > 0, fk, kind)
    return kind


def face_midpoints(mesh, cells, k):
    """Midpoint (x, y) of face k of the given cells (vertex k to k + 1)."""
    cn = np.asarray(mesh.cell_nodes)[np.asarray(cells)]
    nf = np.where(cn[..., 3] < 0, 3, 4)
    kk = np.minimum(k, nf - 1)
    a = mesh.node_xy[np.take_along_axis(cn, kk[..., None], -1)[..., 0]]
    b = mesh.node_xy[np.take_along_axis(cn, ((kk + 1) % nf)[..., None], -1)[..., 0]]
    m = 0.5 * (a + b)
    return m[..., 0], m[..., 1]


def ghost_state(Wv, kind, nx, ny, inflow=None, fronts=None, pos=None, t=0.0):
    """State outside a boundary face with outward unit normal (nx, ny):
    transmissive - the inner state; reflective - the inner state with its
    normal momentum reversed; inflow s (kind 3 + s) - prescribed state s;
    moving front f (kind 2^16 + f, row f = (ex, ey, c0, s, A, B)) - state A
    where the face midpoint ``pos`` lies behind the line e.x = c0 + s t at
    time t, else state B.  Wv: [V, ...]; kind, nx, ny broadcast against
    Wv[0]."""
    Wv = np.asarray(Wv, dtype=np.float64)
    out = Wv.copy()
    kind = np.broadcast_to(kind, Wv.shape[1:])
    if Wv.shape[0] == 4:
        mn = Wv[1] * nx + Wv[2] * ny
        refl = kind == BC_REFLECTIVE
        out[1] = np.where(refl, Wv[1] - 2.0 * mn * nx, out[1])
        out[2] = np.where(refl, Wv[2] - 2.0 * mn * ny, out[2])
    fixed = (kind >= BC_INFLOW) & (kind < BC_FRONT)
    if inflow is not None and fixed.any():
        idx = np.where(fixed, kind - BC_INFLOW, 0)
        st = np.asarray(inflow, dtype=np.float64)[idx]                     # [..., 4]
        for v in range(Wv.shape[0]):
            out[v] = np.where(fixed, st[..., v], out[v])
    moving = kind >= BC_FRONT
    if fronts is not None and moving.any():
        f = np.asarray(fronts, dtype=np.float64)[np.where(moving, kind - BC_FRONT, 0)]
        behind = f[..., 0] * pos[0] + f[..., 1] * pos[1] < f[..., 2] + f[..., 3] * t
        st = np.where(behind[..., None], f[..., 4:8], f[..., 8:12])
        for v in range(Wv.shape[0]):
            out[v] = np.where(moving, st[..., v], out[v])
    return out


def outside_state(mesh, cells, k, Wv, nx, ny, t=0.0):
    """ghost_state for face k of the given cells of a mesh, at time t."""
    kind = face_kind(mesh, cells, k)
    fronts = getattr(mesh, "fronts", None)
    pos = face_midpoints(mesh, cells, k) if fronts is not None else None
    return ghost_state(Wv, kind, nx, ny, getattr(mesh, "inflow", None), fronts, pos, t)


# --------------------------------------------------------------------------
# characteristic decomposition (Sec. 4, Euler systems)
# --------------------------------------------------------------------------

def roe_average(WL, WR, gamma):
    """Roe's mean state of two conserved states (leading axis = variables):
    density-weighted velocity and total enthalpy, and the sound speed."""
    rL, rR = WL[0], WR[0]
    uL, vL = WL[1] / rL, WL[2] / rL
    uR, vR = WR[1] / rR, WR[2] / rR
    pL = (gamma - 1.0) * (WL[3] - 0.5 * rL * (uL * uL + vL * vL))
    pR = (gamma - 1.0) * (WR[3] - 0.5 * rR * (uR * uR + vR * vR))
    HL, HR = (WL[3] + pL) / rL, (WR[3] + pR) / rR
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    u = (sL * uL + sR * uR) / (sL + sR)
    v = (sL * vL + sR * vR) / (sL + sR)
    H = (sL * HL + sR * HR) / (sL + sR)
    c = np.sqrt((gamma - 1.0) * (H - 0.5 * (u * u + v * v)))
    return u, v, H, c


def eigenvectors(u, v, H, c, nx, ny, gamma):
    """Right eigenvectors (columns of R) and left eigenvectors (rows of
    R^-1) of n_x dF/dW + n_y dG/dW for the 2D Euler equations at the state
    (u, v, H, c); eigenvalues u.n - c, u.n, u.n, u.n + c.  Returns
    (R, Rinv, lam) with shapes [..., 4, 4], [..., 4, 4], [..., 4]."""
    un = u * nx + v * ny
    ut = -u * ny + v * nx
    q2 = 0.5 * (u * u + v * v)
    one, zero = np.ones_like(u), np.zeros_like(u)
    R = np.stack([
        np.stack([one, u - c * nx, v - c * ny, H - c * un], -1),
        np.stack([one, u, v, q2], -1),
        np.stack([zero, -ny * one, nx * one, ut], -1),
        np.stack([one, u + c * nx, v + c * ny, H + c * un], -1),
    ], -1)                                                   # columns are eigenvectors
    b1 = (gamma - 1.0) / (c * c)
    b2 = q2 * b1
    Rinv = np.stack([
        np.stack([0.5 * (b2 + un / c), 0.5 * (-b1 * u - nx / c), 0.5 * (-b1 * v - ny / c),
                  0.5 * b1], -1),
        np.stack([1.0 - b2, b1 * u, b1 * v, -b1], -1),
        np.stack([-ut, -ny * one, nx * one, zero], -1),
        np.stack([0.5 * (b2 - un / c), 0.5 * (-b1 * u + nx / c), 0.5 * (-b1 * v + ny / c),
                  0.5 * b1], -1),
    ], -2)                                                   # rows are left eigenvectors
    lam = np.stack([un - c, un, un, un + c], -1)
    return R, Rinv, lam


# --------------------------------------------------------------------------
# reconstruction (WENO or linear) at the Gauss points of a group of cells
# --------------------------------------------------------------------------

def split_linear_weights(gam, theta):
    """Split of the optimised linear weights (Sec. 3.4) along the last axis:
    gamma~+ = (gamma + theta |gamma|)/2, gamma~- = gamma~+ - gamma, their
    sums sigma^pm, and the scaled non-negative weights gamma^pm =
    gamma~pm / sigma^pm.  Returns (gamma^+, sigma^+, gamma^-, sigma^-), the
    sums with a kept last axis of length one."""
    gam = np.asarray(gam, dtype=np.float64)
    tp = 0.5 * (gam + theta * np.abs(gam))
    tm = tp - gam
    sp = tp.sum(axis=-1, keepdims=True)
    sm = tm.sum(axis=-1, keepdims=True)
    return tp / sp, sp, tm / sm, sm


def new_smoothness_indicator(beta, gw):
    """The smoothness indicator of Sec. 3.4 that takes the linear weight into
    account: beta~ = beta (1 + gamma beta + (gamma beta)^2), gamma one of the
    scaled split weights gamma^pm of the candidate."""
    t = gw * beta
    return beta * (1.0 + t + t * t)


def nonlinear_weights(gw, beta, eps):
    """delta_j = alpha_j / sum_l alpha_l with alpha_j = gamma_j / (beta~_j +
    eps)^2 (Sec. 3.4), over the last axis (the candidates)."""
    alpha = gw / (new_smoothness_indicator(beta, gw) + eps) ** 2
    return alpha / alpha.sum(axis=-1, keepdims=True)


def _nonlinear_combination(gp, sp, gm, sm, beta, d, eps):
    """sum over signs of sign sigma^pm sum_j delta_j^pm d_j, with the new
    smoothness indicator of Sec. 3.4.  gp, gm: [m,G,M] normalised split
    weights; sp, sm: [m,G,1] their sums; beta: [F,m,G,M] indicators;
    d: [F,m,G,M] candidate increments P_j(x_G) - W_i0 (F fields)."""
    out = 0.0
    for gw, sig, sgn in ((gp, sp, 1.0), (gm, sm, -1.0)):
        delta = nonlinear_weights(gw[None], beta, eps)
        out = out + sgn * sig[None, :, :, 0] * (delta * d).sum(axis=-1)
    return out                                          # [F,m,G]


def candidate_gradients(g, dW, rows):
    """Gradients and smoothness indicators of the linear candidates (Sec. 3.1,
    3.2, 3.4) of the given rows of a cell group, from the stencil differences
    dW [V,m,S] (dW[..., s] = W of stencil slot s minus W_i0).  Candidate j
    over {i0, a, b} has, in the scaled frame of the target cell, the
    gradient g_j = Y_j (dW_a, dW_b).  With K = 1 the indicator of Sec. 3.4 is
    beta_j = int_Omega |grad P_j|^2 = |Omega| |grad P_j|^2 (the gradient of a
    linear P is constant), and in coordinates scaled by sqrt|Omega| the
    gradient is g_j = sqrt|Omega| grad P_j, so beta_j = |g_j|^2.
    Returns gx, gy, beta, each [V,m,M]."""
    Y = g.Y[rows]                                       # [m,M,2,2]
    V, m = dW.shape[0], dW.shape[1]
    M = g.st.spec.M
    dWa = dW[:, :, g.cand_a]                            # [V,m,M]
    dWb = np.take_along_axis(dW, np.broadcast_to(g.cand_b[rows][None], (V, m, M)), axis=2)
    gx = Y[None, :, :, 0, 0] * dWa + Y[None, :, :, 0, 1] * dWb
    gy = Y[None, :, :, 1, 0] * dWa + Y[None, :, :, 1, 1] * dWb
    return gx, gy, gx * gx + gy * gy


def _weno_group(g, W, scheme, rows, gamma=1.4, mesh=None, t=0.0):
    st = g.st
    cells = st.cells[rows]
    rc = st.runtime_cell[rows]                          # [m,S]
    W0 = W[:, cells]                                    # [V,m]
    dW = W[:, rc] - W0[:, :, None]                      # [V,m,S]
    # ghost face neighbours carry the outside state of their face
    gh = st.ghost[rows]
    for k in range(st.spec.n):
        b = gh[:, k + 1] >= 0
        if mesh is None or not b.any():
            continue
        nrm = g.normal[rows][:, k]
        ghost = outside_state(mesh, cells, k, W0, nrm[:, 0], nrm[:, 1], t)
        dW[:, :, k + 1] = np.where(b[None], ghost - W0, dW[:, :, k + 1])
    off = g.gp_off[rows]                                # [m,G,2]
    if scheme.mode == "linear":
        eta = g.eta[rows]                               # [m,G,S]
        return W0[:, :, None] + np.einsum("mgs,vms->vmg", eta[:, :, 1:], dW[:, :, 1:])
    gx, gy, beta = candidate_gradients(g, dW, rows)      # [V,m,M]
    gp, sp, gm, sm = split_linear_weights(g.gamma[rows], scheme.theta)   # [m,G,M], [m,G,1]
    G = gp.shape[1]
    # P_j(x_G) - W_i0 at every point: [V,m,G,M]
    d = off[None, :, :, None, 0] * gx[:, :, None, :] + off[None, :, :, None, 1] * gy[:, :, None, :]
    if scheme.variables == "characteristic" and W.shape[0] == 4:
        # projection of each Gauss point: Roe mean of the cell and the
        # neighbour across the point's face, with that face's normal
        face = np.arange(G) // 2
        Wnb = W0[:, :, None] + dW[:, :, 1 + face]       # [V,m,G] face neighbour or ghost
        u, v, H, c = roe_average(W0[:, :, None], Wnb, gamma)
        nrm = g.normal[rows][:, face]                   # [m,G,2]
        Rm, Li, _ = eigenvectors(u, v, H, c, nrm[..., 0], nrm[..., 1], gamma)   # [m,G,4,4]
        dc = np.einsum("mgcv,vmgj->cmgj", Li, d)
        gxc = np.einsum("mgcv,vmj->cmgj", Li, gx)
        gyc = np.einsum("mgcv,vmj->cmgj", Li, gy)
        inc = _nonlinear_combination(gp, sp, gm, sm, gxc * gxc + gyc * gyc, dc, scheme.eps)
        return W0[:, :, None] + np.einsum("mgvc,cmg->vmg", Rm, inc)
    inc = _nonlinear_combination(gp, sp, gm, sm, np.broadcast_to(beta[:, :, None, :], d.shape),
                                 d, scheme.eps)
    return W0[:, :, None] + inc                         # [V,m,G]


def reconstruct_face_states(tables: Tables, W, cells=None, gamma=1.4, t=0.0):
    """Reconstructed values at the 2n Gauss points of each requested cell.

    Returns a dict cell -> array [V, 2n] (point g = 2k + q is the q-th Gauss
    point of face k, ordered from v_k to v_{k+1})."""
    W = np.asarray(W, dtype=np.float64)
    if cells is None:
        cells = np.flatnonzero(tables.loc >= 0)
    cells = np.asarray(cells, dtype=np.int64)
    out = {}
    for nf_value, g in tables.groups.items():
        loc = tables.loc[cells]
        mine = cells[(loc >> 32) == nf_value]
        if mine.size == 0:
            continue
        rows = (tables.loc[mine] & 0xFFFFFFFF).astype(np.int64)
        step = 8192
        for i in range(0, rows.size, step):
            R = _weno_group(g, W, tables.scheme, rows[i:i + step], gamma, tables.mesh, t)
            for c, r in zip(mine[i:i + step], np.moveaxis(R, 1, 0)):
                out[int(c)] = r
    return out


# --------------------------------------------------------------------------
# fluxes
# --------------------------------------------------------------------------

def physical_flux(Wv, nx, ny, gamma):
    """Exact Euler flux F(W).n through a face with unit normal (nx, ny)."""
    rho, mu, mv, E = Wv
    u, v = mu / rho, mv / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    un = u * nx + v * ny
    return np.stack([rho * un, mu * un + p * nx, mv * un + p * ny, (E + p) * un])


def hllc_flux(WL, WR, nx, ny, gamma):
    """HLLC flux for the Euler equations through a face with unit normal
    (nx, ny), from the left state WL to the right state WR ([4, ...] arrays).
    The states are rotated into the face frame (eq. (transform)), the HLLC
    flux is evaluated there, and rotated back."""
    def prim(Wv):
        rho, mu, mv, E = Wv
        un = (mu * nx + mv * ny) / rho
        ut = (-mu * ny + mv * nx) / rho
        p = (gamma - 1.0) * (E - 0.5 * rho * (un * un + ut * ut))
        a = np.sqrt(gamma * p / rho)
        return rho, un, ut, p, E, a

    rL, uL, vL, pL, EL, aL = prim(WL)
    rR, uR, vR, pR, ER, aR = prim(WR)
    SL = np.minimum(uL - aL, uR - aR)
    SR = np.maximum(uL + aL, uR + aR)
    Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) / (rL * (SL - uL) - rR * (SR - uR))

    def flux(r, u, v, p, E):
        return np.stack([r * u, r * u * u + p, r * u * v, (E + p) * u])

    def star(r, u, v, p, E, S):
        c = r * (S - u) / (S - Ss)
        return np.stack([c, c * Ss, c * v, c * (E / r + (Ss - u) * (Ss + p / (r * (S - u))))])

    FL = flux(rL, uL, vL, pL, EL)
    FR = flux(rR, uR, vR, pR, ER)
    UL = np.stack([rL, rL * uL, rL * vL, EL])
    UR = np.stack([rR, rR * uR, rR * vR, ER])
    FsL = FL + SL * (star(rL, uL, vL, pL, EL, SL) - UL)
    FsR = FR + SR * (star(rR, uR, vR, pR, ER, SR) - UR)
    F = np.where(0.0 <= SL, FL, np.where(0.0 <= Ss, FsL, np.where(0.0 < SR, FsR, FR)))
    Fn, Ft = F[1], F[2]
    return np.stack([F[0], Fn * nx - Ft * ny, Fn * ny + Ft * nx, F[3]])


def upwind_flux(uL, uR, nx, ny, ax, ay):
    an = ax * nx + ay * ny
    return np.where(an >= 0.0, an * uL, an * uR)


def _face_flux(physics, WL, WR, nx, ny):
    if physics.equation == "euler":
        return hllc_flux(WL, WR, nx, ny, physics.gamma)
    return upwind_flux(WL, WR, nx, ny, physics.ax, physics.ay)


# --------------------------------------------------------------------------
# residual, time step, RK3
# --------------------------------------------------------------------------

def residual(tables: Tables, W, physics: Physics, cells=None, t=0.0):
    """L(W) = -(1/|Omega_i|) sum_p |l_p| sum_k (1/2) F(x_pk) . n_p for the
    requested cells (default: all).  Returns [V, len(cells)]."""
    W = np.asarray(W, dtype=np.float64)
    conn = tables.conn
    if cells is None:
        cells = np.arange(conn.nf.size)
    cells = np.asarray(cells, dtype=np.int64)
    nb = conn.nbr[cells]
    need = np.unique(np.concatenate([cells, nb[nb >= 0]]))
    R = reconstruct_face_states(tables, W, need, physics.gamma, t)
    V = W.shape[0]
    L = np.zeros((V, cells.size))
    for idx, i in enumerate(cells):
        gi, ri = group_row(tables, int(i))
        acc = np.zeros(V)
        for k in range(int(conn.nf[i])):
            c = int(conn.nbr[i, k])
            Ri = R[int(i)]
            if c < 0:
                nx, ny = gi.normal[ri, k]
                ln = gi.length[ri, k]
                G0 = outside_state(tables.mesh, int(i), k, Ri[:, 2 * k], nx, ny, t)
                G1 = outside_state(tables.mesh, int(i), k, Ri[:, 2 * k + 1], nx, ny, t)
                F0 = _face_flux(physics, Ri[:, 2 * k], G0, nx, ny)
                F1 = _face_flux(physics, Ri[:, 2 * k + 1], G1, nx, ny)
                acc += ln * 0.5 * (F0 + F1)
                continue
            kp = int(conn.nbr_face[i, k])
            Rc = R[c]
            if i < c:      # this cell is the left state
                nx, ny = gi.normal[ri, k]
                ln = gi.length[ri, k]
                F0 = _face_flux(physics, Ri[:, 2 * k], Rc[:, 2 * kp + 1], nx, ny)
                F1 = _face_flux(physics, Ri[:, 2 * k + 1], Rc[:, 2 * kp], nx, ny)
                acc += ln * 0.5 * (F0 + F1)
            else:
                gc, rcr = group_row(tables, c)
                nx, ny = gc.normal[rcr, kp]
                ln = gc.length[rcr, kp]
                F0 = _face_flux(physics, Rc[:, 2 * kp + 1], Ri[:, 2 * k], nx, ny)
                F1 = _face_flux(physics, Rc[:, 2 * kp], Ri[:, 2 * k + 1], nx, ny)
                acc -= ln * 0.5 * (F0 + F1)
        L[:, idx] = -acc / gi.area[ri]
    return L


def residual_vectorized(tables: Tables, W, physics: Physics, t=0.0):
    """Same as ``residual`` for all cells, vectorised over cells per face slot
    (used for large meshes; identical arithmetic per face)."""
    W = np.asarray(W, dtype=np.float64)
    conn = tables.conn
    N = conn.nf.size
    V = W.shape[0]
    R = np.zeros((V, N, 8))
    normal = np.zeros((N, 4, 2))
    length = np.zeros((N, 4))
    area = np.zeros(N)
    for nf_value, g in tables.groups.items():
        cells = g.st.cells
        step = 8192
        for i in range(0, cells.size, step):
            rows = np.arange(i, min(cells.size, i + step))
            R[:, cells[rows], :2 * nf_value] = _weno_group(g, W, tables.scheme, rows,
                                                           physics.gamma, tables.mesh, t)
        normal[cells] = g.normal
        length[cells] = g.length
        area[cells] = g.area
    acc = np.zeros((V, N))
    ids = np.arange(N)
    for k in range(4):
        valid = k < conn.nf
        c = conn.nbr[:, k]
        kp = conn.nbr_face[:, k]
        bnd = valid & (c < 0)
        inn = valid & (c >= 0)
        cc = np.where(inn, c, ids)
        kk = np.where(inn, kp, 0)
        left = ids < cc
        # unused face slots (k >= n) take a valid state; their flux is discarded
        Ri0 = np.where(valid[None], R[:, ids, 2 * k], R[:, ids, 0])
        Ri1 = np.where(valid[None], R[:, ids, 2 * k + 1], R[:, ids, 0])
        nL = np.where((left | bnd)[:, None], normal[:, k], normal[cc, kk])
        nL = np.where(valid[:, None], nL, 1.0 / np.sqrt(2.0))
        # outside of a boundary face: its ghost state
        G0 = outside_state(tables.mesh, ids, k, Ri0, nL[:, 0], nL[:, 1], t)
        G1 = outside_state(tables.mesh, ids, k, Ri1, nL[:, 0], nL[:, 1], t)
        Rc0 = np.where(inn[None], R[:, cc, 2 * kk + 1], G0)    # neighbour value at my point 0
        Rc1 = np.where(inn[None], R[:, cc, 2 * kk], G1)
        lL = np.where(left | bnd, length[:, k], length[cc, kk])
        WL0 = np.where((left | bnd)[None], Ri0, Rc0)
        WR0 = np.where((left | bnd)[None], Rc0, Ri0)
        WL1 = np.where((left | bnd)[None], Ri1, Rc1)
        WR1 = np.where((left | bnd)[None], Rc1, Ri1)
        F0 = _face_flux(physics, WL0 if V > 1 else WL0[0], WR0 if V > 1 else WR0[0], nL[:, 0], nL[:, 1])
        F1 = _face_flux(physics, WL1 if V > 1 else WL1[0], WR1 if V > 1 else WR1[0], nL[:, 0], nL[:, 1])
        F0 = np.reshape(F0, (V, N))
        F1 = np.reshape(F1, (V, N))
        s = np.where(left | bnd, 1.0, -1.0)
        contrib = lL * 0.5 * (F0 + F1) * s
        acc += np.where(valid[None], contrib, 0.0)
    return -acc / area[None, :]


def cfl_dt(tables: Tables, W, physics: Physics, cfl: float):
    """CFL-limited time step from cell averages."""
    W = np.asarray(W, dtype=np.float64)
    best = np.inf
    for g in tables.groups.values():
        cells = g.st.cells
        if physics.equation == "euler":
            rho, mu, mv, E = W[:, cells]
            u, v = mu / rho, mv / rho
            p = (physics.gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
            c = np.sqrt(physics.gamma * p / rho)
        else:
            u = np.full(cells.size, physics.ax)
            v = np.full(cells.size, physics.ay)
            c = np.zeros(cells.size)
        s = np.zeros(cells.size)
        for k in range(g.st.spec.n):
            un = u * g.normal[:, k, 0] + v * g.normal[:, k, 1]
            s += g.length[:, k] * (np.abs(un) + c)
        best = min(best, float((2.0 * g.area / s).min()))
    return cfl * best


def rk3_step(tables: Tables, W, physics: Physics, dt: float, resid=None, t=0.0, resid_t=None):
    """One step of the three-stage TVD Runge-Kutta scheme of Sec. 4 from
    time t; the stages evaluate time-dependent boundaries at t, t + dt and
    t + dt/2 (the times the stages approximate).  resid(X) or resid_t(X, t)
    replace the scheme's residual (for tests of the integrator alone)."""
    if resid_t is not None:
        r = resid_t
    elif resid is not None:
        def r(X, tt):
            return resid(X)
    else:
        def r(X, tt):
            return residual_vectorized(tables, X, physics, tt)
    Wn = np.asarray(W, dtype=np.float64)
    W1 = Wn + dt * r(Wn, t)
    W2 = 0.75 * Wn + 0.25 * (W1 + dt * r(W1, t + dt))
    return Wn / 3.0 + 2.0 / 3.0 * (W2 + dt * r(W2, t + 0.5 * dt))
