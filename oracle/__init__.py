"""Plain, slow, FP64 CPU oracle of the third-order unstructured WENO scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the library path may import, call or
execute this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library (no kernels, no
headers, no tables); the only common module is ``workloads``, which generates
seeded inputs and contains none of the method's arithmetic.

Every function follows the paper (Zhao, Pan, Wang: "A third-order WENO scheme
on unstructured quadrilateral and triangular meshes") step by step, in FP64
NumPy, with a leading batch axis over cells and no blocking or fusion beyond
what the definitions state.  Where the paper is silent or garbled the reading
taken is stated in the function's docstring.

Modules
-------
mesh       connectivity, validation, space-filling-curve renumbering
stencil    big-stencil slot selection and the candidate sub-stencils (Sec. 3.1, 3.2)
geometry   scaled-frame moments, Gauss points, faces (Sec. 2, 3.1)
weights    regularised least squares, eta, candidates, linear weights,
           optimisation, diagnostics (Sec. 3.1-3.3)
scheme     nonlinear weights, reconstruction, HLLC/upwind flux, residual,
           SSP-RK3, CFL time step (Sec. 2, 3.4, 4)
"""
from .mesh import connectivity, sfc_permutation, hilbert_index, MeshError  # noqa: F401
from .stencil import build_stencils  # noqa: F401
from .weights import precompute, Scheme  # noqa: F401
from .scheme import (residual, rk3_step, cfl_dt, reconstruct_face_states,  # noqa: F401
                     hllc_flux, physical_flux, Physics)
