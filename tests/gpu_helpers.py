"""Shared helpers of the GPU tests and the benchmark: run the HIP path and
the oracle on the same seeded inputs and compare them."""
from __future__ import annotations

import numpy as np

import workloads as wl


def rel_l1(a, b):
    """Largest over variables of sum|a - b| / sum|b|."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    num = np.abs(a - b).sum(axis=-1)
    den = np.maximum(np.abs(b).sum(axis=-1), 1e-300)
    return float((num / den).max())


def max_rel(a, b):
    """Largest over variables of max|a - b| / max|b|: an element-by-element
    bar (one bad element fails it, however many good ones surround it)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    num = np.abs(a - b).max(axis=-1)
    den = np.maximum(np.abs(b).max(axis=-1), 1e-300)
    return float((num / den).max())


# Element-wise bar of the FP64 comparisons: the FP64 linear weights are
# fixed by ill-conditioned least-squares solves (Sec. 3.3), and the library's
# solve (one-sided Jacobi SVD) and the oracle's (LAPACK SVD) agree only to
# about 1e-10 of the largest weight on 30%-jittered meshes
# (test_fp64_tables_match_oracle); where a weight that differs that much
# multiplies a large candidate increment, one residual element moves by up
# to about 1e-11 of the largest.  FP32 rounding dominates that in the FP32
# comparisons, which keep their L1 bar element by element.
FP64_ELEMENT_FACTOR = 100.0


def parity_err(a, b, tol):
    """Relative error in units of the relative-L1 bar ``tol``: the larger of
    the relative L1 difference and the element-wise one (max_rel), the latter
    scaled so that it meets the same ``<= tol`` test at its own bar (tol
    itself for FP32 bars, FP64_ELEMENT_FACTOR x tol for FP64 ones)."""
    elem_tol = FP64_ELEMENT_FACTOR * tol if tol <= 1e-12 else tol
    return max(rel_l1(a, b), max_rel(a, b) * (tol / elem_tol))


def physics_for(uw, equation, precision):
    eq = uw.UW_EULER if equation == "euler" else uw.UW_ADVECTION
    pr = uw.UW_FP64 if precision == "fp64" else uw.UW_FP32
    return uw.make_physics(eq, 1.0, 1.0, 1.4, pr)


def gpu_residual(uw, M, W_orig, equation, precision, device="cuda:0"):
    """L(W) from the HIP library, returned in the original cell order."""
    import torch
    Wi = torch.from_numpy(M.to_internal(W_orig)).to(device)
    L = torch.empty_like(Wi)
    M.residual(physics_for(uw, equation, precision), Wi, L)
    torch.cuda.synchronize()
    return M.to_original(L.cpu().numpy())


def small_meshes():
    return {
        "c1": wl.mesh_c1(),
        "quad": wl.grid_mesh(24, 24, 2.0, 2.0, "quad", 0.2, 2, True),
        "tri": wl.grid_mesh(17, 17, 2.0, 2.0, "tri", 0.2, 3, True),
        "mixed": wl.mesh_c5(n=32, block=8, jitter=0.3, seed=6),
        "sod": wl.mesh_c3(n=40, jitter=0.15, seed=4, band=0.1),
    }
