"""The library's host side against the oracle, without a GPU: exported
symbols, the Hilbert permutation and stencils (bit-exact), the FP64
precompute tables, and the error paths of the C-ABI."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as wl
from oracle import mesh as om
from oracle import stencil as ost
from oracle import weights as ow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def uw():
    import paper_1712_08317_amd as mod
    return mod


def test_library_exports_every_declared_symbol(uw):
    header = open(os.path.join(ROOT, "include", "uweno.h")).read()
    declared = set(re.findall(r"\b(uw_[a-z0-9_]+)\s*\(", header))
    lib = ctypes.CDLL(uw.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(uw.EXPORTS)


MESHES = {
    "quad": lambda: wl.grid_mesh(12, 12, 2.0, 2.0, "quad", 0.25, 21, True),
    "tri": lambda: wl.grid_mesh(10, 10, 2.0, 2.0, "tri", 0.3, 22, True),
    "mixed": lambda: wl.mesh_c5(n=32, block=8, jitter=0.3, seed=23),
    "sod": lambda: wl.mesh_c3(n=30, jitter=0.15, seed=24, band=0.1),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_permutation_and_stencils_bit_exact(uw, name):
    mesh = MESHES[name]()
    M = uw.Mesh.from_workload(mesh, device=-1)
    new_of_old, _ = om.sfc_permutation(mesh)
    assert np.array_equal(M.new_of_old, new_of_old)
    conn = om.connectivity(mesh)
    slots, present, nbr = M.export()
    assert M.n_interior_faces == int((conn.nbr >= 0).sum()) // 2
    # face neighbours
    lib_nbr = np.where(nbr >= 0, M.old_of_new[np.maximum(nbr, 0)], -1)[M.new_of_old]
    valid = np.arange(4)[None] < conn.nf[:, None]
    assert np.array_equal(np.where(valid, lib_nbr, -1), np.where(valid, conn.nbr, -1))
    for nf in (4, 3):
        if not (conn.nf == nf).any():
            continue
        st = ost.build_stencils(mesh, conn, nf)
        rows = M.new_of_old[st.cells]
        S = st.spec.S
        assert np.array_equal(M.old_of_new[slots[rows, :S]], st.runtime_cell)
        assert np.array_equal(present[rows, :S].astype(bool), st.present)


@pytest.mark.parametrize("name", list(MESHES))
def test_fp64_tables_match_oracle(uw, name):
    mesh = MESHES[name]()
    M = uw.Mesh.from_workload(mesh, device=-1)
    d = M.precompute()
    T = ow.precompute(mesh)
    od = ow.diagnostics(T)
    assert d["n_absent_slots"] == od["n_absent_slots"]
    assert abs(d["max_abs_gamma_opt"] / od["max_abs_gamma_opt"] - 1) < 1e-9
    gam, eta, Y, off, face = (M.table(k) for k in (0, 1, 2, 3, 4))
    for nf, g in T.groups.items():
        rows = M.new_of_old[g.st.cells]
        G, Mc, S = 2 * nf, g.st.spec.M, g.st.spec.S
        scale = max(1.0, np.abs(g.gamma).max())
        assert np.abs(gam[rows][:, :G, :Mc] - g.gamma).max() < 1e-10 * scale
        assert np.abs(eta[rows][:, :G, :S] - g.eta).max() < 1e-11
        assert np.abs(Y[rows][:, :Mc].reshape(-1, Mc, 2, 2) - g.Y).max() < 1e-11
        assert np.abs(off[rows][:, :G] - g.gp_off).max() < 1e-13
        # face scale |l| / (2 |Omega|) of the cell's own faces
        coef = g.length[:, :nf] / (2 * g.area[:, None])
        assert np.allclose(face[rows][:, :nf, 2], coef, rtol=1e-13)


def _desc(uw, xy, cells, bc=1):
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    return xy, cells


@pytest.mark.parametrize("cells,xy,bc", [
    ([[0, 2, 1, -1]], [[0, 0], [1, 0], [0, 1]], 1),                         # clockwise
    ([[0, 1, 2, -1], [0, 1, 3, -1]], [[0, 0], [1, 0], [0, 1], [1, 1]], 1),    # same-direction edge
    ([[0, 1, 2, -1], [1, 0, 3, -1], [1, 0, 4, -1]],
     [[0, 0], [1, 0], [0.5, 1], [0.5, -1], [0.2, -2]], 1),                  # three owners
    ([[0, 1, 1, -1]], [[0, 0], [1, 0], [0, 1]], 1),                          # repeated node
    ([[0, 1, 7, -1]], [[0, 0], [1, 0], [0, 1]], 1),                          # node out of range
    ([[0, 1, 2, -1]], [[0, 0], [1, 0], [0, 1]], 0),                          # unmatched, periodic
])
def test_invalid_meshes_are_rejected(uw, cells, xy, bc):
    with pytest.raises(uw.UwError) as e:
        uw.Mesh(np.array(xy, float), np.array(cells, np.int32), None, bc, device=-1)
    assert e.value.status == uw.UW_EMESH


def test_call_order_and_arguments(uw):
    mesh = wl.grid_mesh(4, 4, 1.0, 1.0, "quad", 0.0, 1, True)
    M = uw.Mesh.from_workload(mesh, device=-1)
    ph = uw.make_physics()
    W = np.zeros((4, M.n_cells))
    L = np.zeros_like(W)
    with pytest.raises(uw.UwError) as e:
        M.residual(ph, W, L, stream=0)
    assert e.value.status == uw.UW_ESTATE
    with pytest.raises(uw.UwError) as e:
        M.table(0)
    assert e.value.status == uw.UW_ESTATE
    with pytest.raises(uw.UwError) as e:
        M.precompute(uw.make_scheme(eps=-1.0))
    assert e.value.status == uw.UW_EINVAL
    with pytest.raises(uw.UwError) as e:
        M.precompute(uw.make_scheme(variables=5))
    assert e.value.status == uw.UW_EINVAL
    M.precompute()
    with pytest.raises(uw.UwError) as e:        # host-only mesh
        M.residual(ph, W, L, stream=0)
    assert e.value.status == uw.UW_ESTATE
    with pytest.raises(uw.UwError) as e:        # host-only mesh, no-allocation variant
        M.residual_noalloc(ph, W, L, stream=0)
    assert e.value.status == uw.UW_ESTATE
    bad = uw.make_physics(equation=7)
    with pytest.raises(uw.UwError) as e:
        M.residual(bad, W, L, stream=0)
    assert e.value.status == uw.UW_EINVAL
    with pytest.raises(uw.UwError) as e:
        M.residual_noalloc(bad, W, L, stream=0)
    assert e.value.status == uw.UW_EINVAL
    st = uw.LIB.uw_mesh_upload(None, -1, None)
    assert st == uw.UW_EINVAL


def test_diagnostics_report_optimisation(uw):
    mesh = wl.grid_mesh(16, 16, 2.0, 2.0, "tri", 0.3, 7, True)
    M = uw.Mesh.from_workload(mesh, device=-1)
    d = M.precompute()
    assert d["max_abs_gamma_raw"] > 50 * d["max_abs_gamma_opt"]
    assert d["max_abs_gamma_opt"] < 12 and d["resid_opt"] < 1e-9
    d0 = M.precompute(uw.make_scheme(optimize=False))
    assert d0["max_abs_gamma_opt"] == pytest.approx(d["max_abs_gamma_raw"], rel=1e-9)


def test_boundary_kinds_are_validated(uw):
    mesh = wl.box_mesh(wl.BC_REFLECTIVE, n=6)
    M = uw.Mesh.from_workload(mesh, device=-1)
    M.precompute()
    bad = mesh.face_bc.copy()
    bad[:] = 7                                   # inflow state 4 of none
    with pytest.raises(uw.UwError) as e:
        uw.Mesh(mesh.node_xy, mesh.cell_nodes, None, uw.UW_BC_TRANSMISSIVE, device=-1,
                face_bc=bad)
    assert e.value.status == uw.UW_EINVAL
    # with the state given it is accepted
    uw.Mesh(mesh.node_xy, mesh.cell_nodes, None, uw.UW_BC_TRANSMISSIVE, device=-1,
            face_bc=np.full_like(bad, uw.UW_BC_INFLOW), inflow=np.ones((1, 4)))
    # an unmatched face left periodic is not a mesh
    per = mesh.face_bc.copy()
    per[:] = 0
    with pytest.raises(uw.UwError) as e:
        uw.Mesh(mesh.node_xy, mesh.cell_nodes, None, uw.UW_BC_PERIODIC, device=-1, face_bc=per)
    assert e.value.status == uw.UW_EMESH
    # the stencils do not depend on the kinds
    M2 = uw.Mesh(mesh.node_xy, mesh.cell_nodes, None, uw.UW_BC_TRANSMISSIVE, device=-1)
    assert all(np.array_equal(a, b) for a, b in zip(M.export(), M2.export()))


def test_front_kinds_are_validated(uw):
    mesh, _ = wl.double_mach(nx=8, ny=2)
    # accepted as built
    uw.Mesh.from_workload(mesh, device=-1)
    args = (mesh.node_xy, mesh.cell_nodes, None, uw.UW_BC_TRANSMISSIVE)
    # a front index past the list
    bad = np.where(mesh.face_bc >= uw.UW_BC_FRONT, uw.UW_BC_FRONT + 1, mesh.face_bc)
    for kw in (dict(face_bc=bad, inflow=mesh.inflow, fronts=mesh.fronts),
               dict(face_bc=mesh.face_bc, inflow=mesh.inflow),               # no fronts at all
               dict(face_bc=mesh.face_bc, inflow=mesh.inflow,
                    fronts=np.where(np.arange(12) == 5, np.nan, mesh.fronts)),   # not finite
               dict(face_bc=mesh.face_bc, inflow=np.ones((65534, 4)), fronts=mesh.fronts)):
        with pytest.raises(uw.UwError) as e:
            uw.Mesh(*args, device=-1, **kw)
        assert e.value.status == uw.UW_EINVAL, kw.keys()
    # prescribed states up to the front kinds are accepted
    uw.Mesh(*args, device=-1, face_bc=mesh.face_bc, inflow=np.ones((65533, 4)),
            fronts=mesh.fronts)


def test_split_parameter_must_exceed_one(uw):
    """theta = 1 leaves the negative part of an all-positive weight set
    empty (0/0 in its normalisation): rejected."""
    mesh = wl.grid_mesh(6, 6, 1.0, 1.0, "quad", 0.1, 1, True)
    M = uw.Mesh.from_workload(mesh, device=-1)
    with pytest.raises(uw.UwError) as e:
        M.precompute(uw.make_scheme(theta=1.0))
    assert e.value.status == uw.UW_EINVAL
    M.precompute(uw.make_scheme(theta=1.5))


def test_c_abi_from_plain_c(uw, tmp_path):
    """include/uweno.h compiles as C99 and a C program linked against the
    library uploads, precomputes and inspects a host-only mesh."""
    import shutil
    import subprocess
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = tmp_path / "c_abi_check"
    libdir = os.path.dirname(uw.LIB_PATH)
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi_check.c"), "-o", str(exe), "-L", libdir,
                    "-luweno", "-Wl,-rpath," + libdir], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
