"""Edge cases of the method and of the interface: empty input, one cell,
periodic meshes so small that a cell's stencil wraps onto itself (and the
ones too small to be a mesh), ragged last tiles, a triangle alone among
quadrilaterals, and a batch holding a one-cell instance.  The CPU tests
check that library and oracle accept and reject the same inputs; the GPU
tests compare results with the oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle import mesh as om
from oracle import weights as ow
from oracle import scheme as osc
from gpu_helpers import gpu_residual, parity_err, physics_for


@pytest.fixture(scope="module")
def uw():
    import paper_1712_08317_amd as mod
    return mod


def test_empty_mesh_is_rejected(uw):
    with pytest.raises(uw.UwError) as e:
        uw.Mesh(np.zeros((0, 2)), np.zeros((0, 4), np.int32), None, uw.UW_BC_TRANSMISSIVE,
                device=-1)
    assert e.value.status == uw.UW_EINVAL


@pytest.mark.parametrize("n,kind", [(1, "quad"), (2, "quad"), (1, "tri"), (2, "tri")])
def test_periodic_meshes_too_small_are_rejected_by_both(uw, n, kind):
    """One or two squares per period identify a cell's edge with itself or
    give an edge more than two owners: not a mesh, for either side."""
    mesh = wl.grid_mesh(n, n, 2.0, 2.0, kind, 0.0, 1, True)
    with pytest.raises(om.MeshError):
        om.connectivity(mesh)
    with pytest.raises(uw.UwError) as e:
        uw.Mesh.from_workload(mesh, device=-1)
    assert e.value.status == uw.UW_EMESH


def _single(kind):
    if kind == "quad":
        xy = np.array([[0.0, 0.0], [1.0, 0.1], [1.1, 1.0], [-0.1, 0.9]])
        cells = np.array([[0, 1, 2, 3]], np.int32)
    else:
        xy = np.array([[0.0, 0.0], [1.0, 0.2], [0.3, 0.9]])
        cells = np.array([[0, 1, 2, -1]], np.int32)
    # with open faces only, a lone cell's residual vanishes for any state (all
    # outside states are the cell's own); an inflow face and a wall make it
    # a real test
    face_bc = np.array([[wl.BC_INFLOW, wl.BC_REFLECTIVE, wl.BC_TRANSMISSIVE, wl.BC_REFLECTIVE]],
                       np.int32)
    return wl.Mesh(node_xy=xy, cell_nodes=cells, node_id=None, period=(0.0, 0.0),
                   bc="transmissive", h=1.0, name=f"single-{kind}", face_bc=face_bc,
                   inflow=wl.primitive_to_conserved(1.2, 0.5, 0.1, 1.3)[None, :])


def _ragged(nx, ny):
    # nx * ny - 1 quadrilaterals and one split square (two lone triangles):
    # the quadrilateral tiles end with a ragged one, the triangle tile holds 2
    split = np.zeros((ny, nx), bool)
    split[ny // 2, nx // 2] = True
    return wl.grid_mesh(nx, ny, 2.0 * nx / ny, 2.0, split, 0.2, 60 + nx, True,
                        name=f"ragged{nx}x{ny}")


@pytest.mark.parametrize("kind", ["quad", "tri"])
def test_single_cell_precompute_matches_oracle(uw, kind):
    mesh = _single(kind)
    M = uw.Mesh.from_workload(mesh, device=-1)
    d = M.precompute()
    T = ow.precompute(mesh)
    assert d["n_absent_slots"] == ow.diagnostics(T)["n_absent_slots"]


GPU_CASES = {
    "single-quad": lambda: _single("quad"),
    "single-tri": lambda: _single("tri"),
    "periodic-3x3-quad": lambda: wl.grid_mesh(3, 3, 2.0, 2.0, "quad", 0.2, 7, True),
    "periodic-3x3-tri": lambda: wl.grid_mesh(3, 3, 2.0, 2.0, "tri", 0.2, 8, True),
    "ragged-257q": lambda: _ragged(86, 3),      # 257 quads + 2 triangles
    "ragged-511q": lambda: _ragged(128, 4),     # 511 quads + 2 triangles
}


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(GPU_CASES))
@pytest.mark.parametrize("prec,tile", [("fp64", 256), ("fp32", 256), ("fp32", 512)])
def test_edge_case_residual_matches_oracle(uw, name, prec, tile):
    mesh = GPU_CASES[name]()
    M = uw.Mesh.from_workload(mesh, device=0)
    M.precompute()
    M.tile_size(tile)
    T = ow.precompute(mesh)
    W = wl.seeded_state(mesh, 4, 71)
    ref = osc.residual_vectorized(T, W, osc.Physics("euler"))
    got = gpu_residual(uw, M, W, "euler", prec)
    tol = 1e-12 if prec == "fp64" else 1e-5
    err = parity_err(got, ref, tol)
    print(name, prec, tile, mesh.n_cells, "cells, rel L1 / elementwise", err)
    assert err <= tol
    # a uniform state gives a residual at rounding level (without walls or
    # prescribed states, which act on it)
    if mesh.face_bc is None:
        U = np.tile(np.array([[1.1], [0.3], [-0.2], [2.7]]), (1, mesh.n_cells))
        tol = 1e-12 if prec == "fp64" else 1e-4
        assert np.abs(gpu_residual(uw, M, U, "euler", prec)).max() < tol


@pytest.mark.gpu
def test_batch_with_a_one_cell_instance(uw):
    import torch
    meshes = [_single("quad"), wl.grid_mesh(20, 20, 2.0, 2.0, "tri", 0.2, 72, True), _single("tri"),
              _ragged(86, 3)]
    Ms = [uw.Mesh.from_workload(m, device=0) for m in meshes]
    for M in Ms:
        M.precompute()
    states = [wl.seeded_state(m, 4, 73 + k) for k, m in enumerate(meshes)]
    ph = physics_for(uw, "euler", "fp64")
    B = uw.Batch(Ms, ph)
    Wb = torch.from_numpy(B.to_internal(states)).to("cuda:0")
    tb = torch.zeros(len(Ms), dtype=torch.float64, device="cuda:0")
    dt = 1e-3
    B.rk3_step(Wb, tb, dt_fixed=dt, n_steps=2)
    B.check()
    got = B.to_original(Wb.cpu().numpy())
    for k, mesh in enumerate(meshes):
        T = ow.precompute(mesh)
        ref = states[k]
        for _ in range(2):
            ref = osc.rk3_step(T, ref, osc.Physics("euler"), dt)
        assert parity_err(got[k], ref, 1e-12) <= 1e-12, k
