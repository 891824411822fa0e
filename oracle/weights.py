"""Oracle: least squares, linear weights, their optimisation and diagnostics.

Test infrastructure only (see the package docstring).

Paper, Sec. 3.1-3.3:
* eq. (quadratic-2): the regularised least squares (zeta I + A^T A) a = A^T dW
  with zeta = 1e-14, and its weighted form for the optimisation (rows scaled
  by d_j);
* eq. (polynomial-eta): P^2(x_G) = sum_j eta_j W_ij with eta_j = 0 where E_j = 0;
* the candidate linear polynomials P^1_j on the sub-stencils, written as
  P^1_j(x_G) = sum_k b_jk W_Sjk (with the substituted cell for absent slots);
* eq. (linearweight-matrix): B gamma = eta, solved by the same regularised
  least squares (zeta I + B^T B) gamma = B^T eta;
* Sec. 3.3: d_j = 1/max(1,|gamma_j|) (quadrilaterals, j = 5..12) or
  1/max(1,|gamma_j|,|gamma_k|) over the listed pairs (triangles), then the
  weighted quadratic and the optimised gamma.

Readings:
* the regularised normal equations are evaluated through the singular value
  decomposition, x = V diag(s/(s^2 + zeta)) U^T r, which is the same
  Tikhonov solution without squaring the condition number (B has rank 11 for
  a quadrilateral; its zeta -> 0 limit is the minimum-norm solution);
* the candidate fit keeps the zero-mean form W_i0 + g . (p^1, p^2), so the
  constraint on i0 holds exactly and the two remaining constraints give a
  2x2 regularised solve g = Y (dW_a, dW_b);
* the optimisation weights are taken per Gauss point from that point's
  unoptimised gamma (one pass, not iterated);
* optimised weights of magnitude below 1e-10 are set to zero.  Such weights
  arise for degenerate candidates (whose third cell is the target cell after
  substitution, next to a boundary) as the rounding residue of O(1) terms,
  with no significant digit; kept, a rounding-level weight on a candidate
  whose indicator is zero (a field that is constant across a wall, say)
  outweighs every other candidate and the result follows the rounding.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .geometry import Frame, face_geometry
from .mesh import connectivity
from .stencil import build_stencils


@dataclasses.dataclass
class Scheme:
    zeta: float = 1e-14
    theta: float = 3.0
    eps: float = 1e-3
    optimize: bool = True
    d_scope: str = "gp"       # "gp": d per Gauss point; "cell": from max over the cell's points
    mode: str = "weno"        # "weno" or "linear"
    variables: str = "conserved"   # "conserved" or "characteristic" (Euler only)


RANK_TOL = 1e-12
# linear weights below this magnitude are zero: formed from O(1) quantities,
# they carry no significant digit (degenerate candidates next to boundaries)
GAMMA_ZERO = 1e-10


def tikhonov(Mat, zeta):
    """X = (zeta I + M^T M)^{-1} M^T evaluated as V diag(s/(s^2+zeta)) U^T.

    Singular values below RANK_TOL * s_max are rounding noise of an exactly
    rank-deficient matrix (a stencil with too few cells, or the two linear
    identities that make B rank-deficient); in exact arithmetic M^T removes
    those directions, so their filter factor is set to zero."""
    U, s, Vh = np.linalg.svd(Mat, full_matrices=False)
    f = s / (s * s + zeta)
    f = np.where(s > RANK_TOL * s[..., :1], f, 0.0)
    return np.einsum("...ji,...j,...kj->...ik", Vh, f, U)


@dataclasses.dataclass
class Group:
    """Precomputed data of all target cells of one type (3 or 4 faces)."""
    st: object              # Stencils
    frame: object           # Frame
    cand_a: np.ndarray      # [M] slot of the face neighbour of S_j
    cand_b: np.ndarray      # [m,M] slot of the third cell of S_j after substitution
    Y: np.ndarray           # [m,M,2,2] candidate gradient operators, g_j = Y_j (dW_a, dW_b)
    gp_off: np.ndarray      # [m,2n,2] (p^1, p^2) at each Gauss point
    eta: np.ndarray         # [m,2n,S] optimised point-value coefficients of P^2
    gamma: np.ndarray       # [m,2n,M] optimised linear weights
    eta_raw: np.ndarray     # [m,2n,S] before optimisation
    gamma_raw: np.ndarray   # [m,2n,M]
    B: np.ndarray           # [m,2n,S,M]
    length: np.ndarray      # [m,4]
    normal: np.ndarray      # [m,4,2]
    area: np.ndarray        # [m]


@dataclasses.dataclass
class Tables:
    mesh: object
    conn: object
    scheme: Scheme
    groups: dict            # nf -> Group
    loc: np.ndarray         # [N] (nf, row in group) packed as nf*2^32 + row; -1 if not computed


def _group(mesh, conn, nf_value, cells, scheme: Scheme) -> Group:
    st = build_stencils(mesh, conn, nf_value, cells)
    spec = st.spec
    fr = Frame(mesh, st)
    n, S, M = spec.n, spec.S, spec.M
    m = st.cells.size
    zeta = scheme.zeta

    length, normal, gp_xi = face_geometry(fr)
    xiG = gp_xi[:, :n].reshape(m, 2 * n, 2)               # GP index g = 2k + q
    pG = fr.basis_at(xiG)                                 # [m,2n,5]

    # A_jk = E_j <p^k>_{Omega_ij}, j = 1..S-1
    E = st.present[:, 1:].astype(np.float64)
    A = np.where(st.present[:, 1:, None], fr.basis_avg[:, 1:, :], 0.0)

    def eta_of(D):
        """Point-value coefficients of P^2 at every GP with row weights D
        ([m,S-1] shared by all GPs, or [m,2n,S-1] per GP)."""
        # eta_j = 0 where E_j = 0 (eq. (polynomial-eta)): the zero rows of A
        # give zero columns of (zeta I + A^T A)^{-1} A^T
        if D.ndim == 2:
            X = tikhonov(D[:, :, None] * A, zeta) * (D * E)[:, None, :]    # [m,5,S-1]
            e = np.einsum("mgk,mkj->mgj", pG, X)
        else:
            DA = D[..., None] * A[:, None]                                 # [m,2n,S-1,5]
            X = tikhonov(DA, zeta) * (D * E[:, None, :])[:, :, None, :]    # [m,2n,5,S-1]
            e = np.einsum("mgk,mgkj->mgj", pG, X)
        e0 = 1.0 - e.sum(axis=-1, keepdims=True)
        return np.concatenate([e0, e], axis=-1)                            # [m,2n,S]

    eta_raw = eta_of(np.ones((m, S - 1)))

    # candidates: S_j = {i0, a_j, b_j}; the third cell after substitution
    cand_a = np.array([a for a, _ in spec.sub])
    cand_b = np.stack([st.resolved[:, b] for _, b in spec.sub], axis=1)    # [m,M]
    rows_a = fr.basis_avg[:, cand_a, :2]                                   # [m,M,2]
    rows_b = np.take_along_axis(fr.basis_avg[:, :, :2], cand_b[:, :, None], axis=1)
    Mj = np.stack([rows_a, rows_b], axis=2)                                # [m,M,2(rows),2]
    Y = tikhonov(Mj, zeta)                                                 # [m,M,2,2]

    # b_jk(G): coefficients of W_i0, W_a, W_b in P^1_j(x_G)
    off = pG[..., :2]                                                      # [m,2n,2]
    b_ab = np.einsum("mgc,mjcr->mgjr", off, Y)                             # [m,2n,M,2]
    B = np.zeros((m, 2 * n, S, M))
    mi = np.arange(m)[:, None]
    for j in range(M):
        B[:, :, 0, j] += 1.0 - b_ab[:, :, j, 0] - b_ab[:, :, j, 1]
        B[:, :, cand_a[j], j] += b_ab[:, :, j, 0]
        B[mi, np.arange(2 * n)[None, :], cand_b[:, j][:, None], j] += b_ab[:, :, j, 1]
    PB = tikhonov(B, zeta)                                                 # [m,2n,M,S]
    gamma_raw = np.einsum("mgjs,mgs->mgj", PB, eta_raw)

    if scheme.optimize:
        mag = np.abs(gamma_raw)                                            # [m,2n,M]
        if scheme.d_scope == "cell":
            mag = np.broadcast_to(mag.max(axis=1, keepdims=True), mag.shape)
        D = np.ones((m, 2 * n, S - 1))
        for slot, cands in spec.d_pairs:
            big = np.ones((m, 2 * n))
            for c in cands:
                big = np.maximum(big, mag[:, :, c - 1])
            D[:, :, slot - 1] = 1.0 / big
        eta = eta_of(D)
        gamma = np.einsum("mgjs,mgs->mgj", PB, eta)
    else:
        eta, gamma = eta_raw, gamma_raw
    # a weight at rounding level would otherwise take over the nonlinear
    # weights wherever its candidate is smooth and the others are not
    gamma = np.where(np.abs(gamma) < GAMMA_ZERO, 0.0, gamma)

    return Group(st=st, frame=fr, cand_a=cand_a, cand_b=cand_b, Y=Y, gp_off=off,
                 eta=eta, gamma=gamma, eta_raw=eta_raw, gamma_raw=gamma_raw, B=B,
                 length=length, normal=normal, area=fr.area)


def precompute(mesh, scheme: Scheme | None = None, cells=None, conn=None,
               chunk: int = 8192) -> Tables:
    """All per-cell precomputed data, for every cell or for a subset."""
    scheme = scheme or Scheme()
    conn = conn if conn is not None else connectivity(mesh)
    n = conn.nf.size
    todo = np.arange(n) if cells is None else np.unique(np.asarray(cells, dtype=np.int64))
    groups = {}
    loc = np.full(n, -1, dtype=np.int64)
    for nf_value in (4, 3):
        sel = todo[conn.nf[todo] == nf_value]
        if sel.size == 0:
            continue
        parts = [_group(mesh, conn, nf_value, sel[i:i + chunk], scheme)
                 for i in range(0, sel.size, chunk)]
        g = parts[0] if len(parts) == 1 else _concat(parts)
        groups[nf_value] = g
        loc[sel] = nf_value * (1 << 32) + np.arange(sel.size)
    return Tables(mesh=mesh, conn=conn, scheme=scheme, groups=groups, loc=loc)


def _concat(parts):
    from .geometry import Frame as _F  # noqa: F401
    from .stencil import Stencils
    st0 = parts[0].st
    st = Stencils(cells=np.concatenate([p.st.cells for p in parts]), spec=st0.spec,
                  cell=np.concatenate([p.st.cell for p in parts]),
                  shift=np.concatenate([p.st.shift for p in parts]),
                  present=np.concatenate([p.st.present for p in parts]),
                  ghost=np.concatenate([p.st.ghost for p in parts]),
                  resolved=np.concatenate([p.st.resolved for p in parts]))
    fr = parts[0].frame
    frame = _ConcatFrame([p.frame for p in parts])
    del fr
    cat = lambda name: np.concatenate([getattr(p, name) for p in parts])  # noqa: E731
    return Group(st=st, frame=frame, cand_a=parts[0].cand_a, cand_b=cat("cand_b"), Y=cat("Y"),
                 gp_off=cat("gp_off"), eta=cat("eta"), gamma=cat("gamma"),
                 eta_raw=cat("eta_raw"), gamma_raw=cat("gamma_raw"), B=cat("B"),
                 length=cat("length"), normal=cat("normal"), area=cat("area"))


class _ConcatFrame:
    def __init__(self, frames):
        for name in ("nf", "area", "centroid", "h0", "raw_polygon", "xi_polygon",
                     "slot_area", "mean0", "basis_avg", "present"):
            setattr(self, name, np.concatenate([getattr(f, name) for f in frames]))


def group_row(tables: Tables, cell: int):
    v = int(tables.loc[cell])
    if v < 0:
        raise KeyError(f"cell {cell} was not precomputed")
    return tables.groups[v >> 32], v & 0xFFFFFFFF


def diagnostics(tables: Tables) -> dict:
    """max|gamma| before and after optimisation, consistency residuals
    ||B gamma - eta||_inf and |sum gamma - 1|, and the absent-slot count."""
    out = dict(max_abs_gamma_raw=0.0, max_abs_gamma_opt=0.0, resid_raw=0.0, resid_opt=0.0,
               sum_dev=0.0, n_absent_slots=0)
    for g in tables.groups.values():
        out["max_abs_gamma_raw"] = max(out["max_abs_gamma_raw"], float(np.abs(g.gamma_raw).max()))
        out["max_abs_gamma_opt"] = max(out["max_abs_gamma_opt"], float(np.abs(g.gamma).max()))
        r1 = np.einsum("mgsj,mgj->mgs", g.B, g.gamma_raw) - g.eta_raw
        r2 = np.einsum("mgsj,mgj->mgs", g.B, g.gamma) - g.eta
        out["resid_raw"] = max(out["resid_raw"], float(np.abs(r1).max()))
        out["resid_opt"] = max(out["resid_opt"], float(np.abs(r2).max()))
        out["sum_dev"] = max(out["sum_dev"], float(np.abs(g.gamma.sum(-1) - 1).max()))
        out["n_absent_slots"] += int((~g.st.present).sum())
    return out
