"""Pins of the oracle's stencil selection (paper Sec. 3.1 and 3.2)."""
import os

import numpy as np
import pytest

import workloads as wl
from oracle import mesh as om
from oracle import stencil as ost

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    out = {}
    for line in open(os.path.join(GOLD, "stencil_uniform.txt")):
        if line.startswith("#") or not line.strip():
            continue
        left, right = line.split("|")
        f = left.split()
        out[f[0]] = (int(f[1]), [int(x) for x in f[2:]], [int(x) for x in right.split()])
    return out


def test_uniform_quad_and_triangle_golden():
    gold = _golden()
    quad = wl.grid_mesh(6, 6, 6.0, 6.0, "quad", 0.0, 1, True)
    tri = wl.grid_mesh(6, 6, 6.0, 6.0, "tri", 0.0, 1, True)
    for name, mesh, nf in (("quad6", quad, 4), ("tri6", tri, 3)):
        target, slots, flags = gold[name]
        conn = om.connectivity(mesh)
        st = ost.build_stencils(mesh, conn, nf, [target])
        assert st.runtime_cell[0].tolist() == slots
        assert st.present[0].astype(int).tolist() == flags


def _brute_slot(mesh, i0, k, end):
    """The cell across the face of face-neighbour i_{k+1} that contains the
    vertex (v_k if end == 0 else v_{k+1}) and is not the face shared with i0,
    found by scanning all cells."""
    cn = mesh.cell_nodes
    canon = np.arange(mesh.n_nodes) if mesh.node_id is None else mesh.node_id
    nf = mesh.n_faces_of()

    def edges(c):
        return [frozenset((canon[cn[c, q]], canon[cn[c, (q + 1) % nf[c]]])) for q in range(nf[c])]

    va, vb = canon[cn[i0, k]], canon[cn[i0, (k + 1) % nf[i0]]]
    shared = frozenset((va, vb))
    owners = [c for c in range(mesh.n_cells) if c != i0 and shared in edges(c)]
    if not owners:
        return None, None
    c = owners[0]
    v = va if end == 0 else vb
    ce = [e for e in edges(c) if v in e and e != shared]
    assert len(ce) == 1
    across = [x for x in range(mesh.n_cells) if x != c and ce[0] in edges(x)]
    return c, (across[0] if across else None)


def _brute_stencil(mesh, i0):
    nf = mesh.n_faces_of()[i0]
    spec = ost.spec_of(nf)
    cells = [i0]
    faces = []
    for k in range(nf):
        c, _ = _brute_slot(mesh, i0, k, 0)
        faces.append(c)
        cells.append(i0 if c is None else c)        # ghost reads i0
    present = [True] * (nf + 1)
    for s_off, (k, end) in enumerate(spec.outer):
        j = nf + 1 + s_off
        c, x = _brute_slot(mesh, i0, k, end)
        ok = x is not None and x != i0 and x not in faces and \
            x not in [cells[q] for q in range(nf + 1, j) if present[q]]
        present.append(ok)
        if ok:
            cells.append(x)
        else:
            # paper: quad i5..i8 -> i0, i9..i12 -> i_{j-4}; tri i4..i6 -> i0, i7..i9 -> i_{j-3}
            first_block = nf + 1 + nf
            cells.append(i0 if j < first_block else cells[j - nf])
    return cells, present


@pytest.mark.parametrize("maker", [
    lambda: wl.grid_mesh(6, 6, 2.0, 2.0, "quad", 0.25, 3, True),
    lambda: wl.grid_mesh(6, 6, 2.0, 2.0, "tri", 0.25, 4, True),
    lambda: wl.mesh_c5(n=12, block=3, jitter=0.3, seed=5),
    lambda: wl.grid_mesh(7, 7, 1.0, 1.0,
                         np.add.outer(np.arange(7), np.arange(7)) % 3 == 0, 0.15, 6, False),
])
def test_slots_match_brute_force(maker):
    mesh = maker()
    conn = om.connectivity(mesh)
    nf = mesh.n_faces_of()
    for nfv in (4, 3):
        ids = np.flatnonzero(nf == nfv)
        if ids.size == 0:
            continue
        st = ost.build_stencils(mesh, conn, nfv, ids)
        for r, i0 in enumerate(ids):
            cells, present = _brute_stencil(mesh, int(i0))
            assert st.runtime_cell[r].tolist() == cells, (i0, st.runtime_cell[r], cells)
            assert st.present[r].tolist() == present


def test_uniform_triangles_have_ten_distinct_cells():
    mesh = wl.grid_mesh(8, 8, 2.0, 2.0, "tri", 0.0, 1, True)
    conn = om.connectivity(mesh)
    st = ost.build_stencils(mesh, conn, 3)
    assert st.present.all()
    for row in st.runtime_cell:
        assert len(set(row.tolist())) == 10


def test_uniform_quads_form_3x3_block():
    n = 8
    mesh = wl.grid_mesh(n, n, 2.0, 2.0, "quad", 0.0, 1, True)
    conn = om.connectivity(mesh)
    st = ost.build_stencils(mesh, conn, 4)
    assert st.present[:, :9].all() and not st.present[:, 9:].any()
    for r, c in enumerate(st.cells):
        i, j = c % n, c // n
        block = {((j + dj) % n) * n + (i + di) % n for di in (-1, 0, 1) for dj in (-1, 0, 1)}
        assert set(st.runtime_cell[r].tolist()) == block


def test_rotating_a_uniform_quad_mesh_permutes_slots_cyclically():
    # renumbering each cell's vertices cyclically (v_k -> v_{k+1}) relabels
    # faces k -> k-1; the big stencil must be the same set of cells with the
    # slot blocks permuted accordingly
    n = 6
    mesh = wl.grid_mesh(n, n, 2.0, 2.0, "quad", 0.0, 1, True)
    rot = wl.Mesh(node_xy=mesh.node_xy, cell_nodes=np.roll(mesh.cell_nodes, -1, axis=1),
                  node_id=mesh.node_id, period=mesh.period, bc=mesh.bc, h=mesh.h)
    a = ost.build_stencils(mesh, om.connectivity(mesh), 4)
    b = ost.build_stencils(rot, om.connectivity(rot), 4)
    for r in range(a.cells.size):
        A, B = a.runtime_cell[r], b.runtime_cell[r]
        assert B[1:5].tolist() == [A[2], A[3], A[4], A[1]]
        assert set(A.tolist()) == set(B.tolist())


def test_transmissive_boundary_ghosts():
    mesh = wl.grid_mesh(4, 4, 1.0, 1.0, "quad", 0.0, 1, False)
    conn = om.connectivity(mesh)
    st = ost.build_stencils(mesh, conn, 4, [0])      # corner cell: faces 0 and 3 on the boundary
    assert st.ghost[0, 1] == 0 and st.ghost[0, 4] == 3
    assert st.runtime_cell[0, 1] == 0 and st.runtime_cell[0, 4] == 0
    assert st.present[0, :5].all()
    # slots reached through the ghosts are absent; i7 (via i3 = cell 4 at v2) is cell 5
    assert st.present[0].tolist() == [1, 1, 1, 1, 1, 0, 0, 1, 0, 0, 0, 0, 0]
    assert st.runtime_cell[0, 7] == 5
