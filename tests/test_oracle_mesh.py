"""Pins of the oracle's connectivity, validation and renumbering."""
import os

import numpy as np
import pytest

import workloads as wl
from oracle import mesh as om

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _brute_neighbours(mesh):
    """O(N^2) search: for every face find the other cell holding the same
    canonical edge in the opposite direction."""
    cn = mesh.cell_nodes
    canon = np.arange(mesh.n_nodes) if mesh.node_id is None else mesh.node_id
    nf = mesh.n_faces_of()
    edges = []
    for c in range(mesh.n_cells):
        for k in range(nf[c]):
            a, b = cn[c, k], cn[c, (k + 1) % nf[c]]
            edges.append((c, k, canon[a], canon[b], a, b))
    nbr = -np.ones((mesh.n_cells, 4), dtype=int)
    nface = -np.ones((mesh.n_cells, 4), dtype=int)
    shift = np.zeros((mesh.n_cells, 4, 2))
    for (c, k, ca, cb, a, b) in edges:
        for (d, kk, da, db, a2, b2) in edges:
            if d != c and da == cb and db == ca:
                nbr[c, k] = d
                nface[c, k] = kk
                shift[c, k] = mesh.node_xy[a] - mesh.node_xy[b2]
    return nbr, nface, shift


@pytest.mark.parametrize("maker", [
    lambda: wl.grid_mesh(5, 5, 2.0, 2.0, "tri", 0.2, 7, True),
    lambda: wl.grid_mesh(6, 5, 2.4, 2.0, "quad", 0.2, 8, True),
    lambda: wl.grid_mesh(6, 6, 1.0, 1.0, np.eye(6, dtype=bool), 0.15, 9, False),
])
def test_connectivity_matches_brute_force(maker):
    mesh = maker()
    conn = om.connectivity(mesh)
    nbr, nface, shift = _brute_neighbours(mesh)
    for c in range(mesh.n_cells):
        for k in range(conn.nf[c]):
            assert conn.nbr[c, k] == nbr[c, k]
            assert conn.nbr_face[c, k] == nface[c, k]
            np.testing.assert_array_equal(conn.shift[c, k], shift[c, k])
    # every interior face is seen exactly twice, with the partner pointing back
    for c in range(mesh.n_cells):
        for k in range(conn.nf[c]):
            d, kk = conn.nbr[c, k], conn.nbr_face[c, k]
            if d >= 0:
                assert conn.nbr[d, kk] == c and conn.nbr_face[d, kk] == k
                np.testing.assert_array_equal(conn.shift[d, kk], -conn.shift[c, k])


def test_shift_places_neighbour_edge_on_cell_edge():
    mesh = wl.grid_mesh(7, 7, 2.0, 2.0, "quad", 0.2, 3, True)
    conn = om.connectivity(mesh)
    cn, xy = mesh.cell_nodes, mesh.node_xy
    for c in range(mesh.n_cells):
        for k in range(4):
            d, kk = conn.nbr[c, k], conn.nbr_face[c, k]
            a, b = xy[cn[c, k]], xy[cn[c, (k + 1) % 4]]
            a2, b2 = xy[cn[d, kk]], xy[cn[d, (kk + 1) % 4]]
            np.testing.assert_array_equal(b2 + conn.shift[c, k], a)
            np.testing.assert_array_equal(a2 + conn.shift[c, k], b)


@pytest.mark.parametrize("kind", ["quad", "tri"])
def test_euler_characteristic_of_periodic_torus(kind):
    mesh = wl.grid_mesh(9, 7, 2.0, 2.0 * 7 / 9, kind, 0.2, 4, True)
    conn = om.connectivity(mesh)
    V = np.unique(mesh.node_id).size
    E = int(((conn.nbr >= 0) & (np.arange(4)[None] < conn.nf[:, None])).sum()) // 2
    F = mesh.n_cells
    assert V - E + F == 0
    assert ((conn.nbr >= 0).sum(axis=1) == conn.nf).all()


def test_open_square_has_boundary_faces():
    mesh = wl.grid_mesh(4, 4, 1.0, 1.0, "quad", 0.0, 1, False)
    conn = om.connectivity(mesh)
    assert int((conn.nbr[:, :4] < 0).sum()) == 16


def _tiny(cells, xy, bc="transmissive"):
    return wl.Mesh(node_xy=np.asarray(xy, float), cell_nodes=np.asarray(cells, np.int32),
                   node_id=None, period=(0.0, 0.0), bc=bc, h=1.0)


def test_rejects_inverted_cell():
    with pytest.raises(om.MeshError):
        om.connectivity(_tiny([[0, 2, 1, -1]], [[0, 0], [1, 0], [0, 1]]))


def test_rejects_edge_with_three_owners():
    xy = [[0, 0], [1, 0], [0.5, 1], [0.5, -1], [0.2, -2]]
    with pytest.raises(om.MeshError):
        om.connectivity(_tiny([[0, 1, 2, -1], [1, 0, 3, -1], [1, 0, 4, -1]], xy))


def test_rejects_same_direction_edge():
    xy = [[0, 0], [1, 0], [0, 1], [1, 1]]
    with pytest.raises(om.MeshError):
        om.connectivity(_tiny([[0, 1, 2, -1], [0, 1, 3, -1]], xy))


def test_rejects_unmatched_face_on_periodic_mesh():
    with pytest.raises(om.MeshError):
        om.connectivity(_tiny([[0, 1, 2, -1]], [[0, 0], [1, 0], [0, 1]], bc="periodic"))


def test_hilbert_order1_sequence():
    d = om.hilbert_index(np.array([0, 0, 1, 1]), np.array([0, 1, 1, 0]), 1)
    assert d.tolist() == [0, 1, 2, 3]


def test_hilbert_order2_golden():
    rows = np.loadtxt(os.path.join(GOLD, "hilbert_order2.txt"), dtype=np.int64)
    d = om.hilbert_index(rows[:, 0], rows[:, 1], 2)
    np.testing.assert_array_equal(d, rows[:, 2])


@pytest.mark.parametrize("order", [3, 5])
def test_hilbert_is_a_continuous_bijection(order):
    n = 1 << order
    x, y = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    d = om.hilbert_index(x.ravel(), y.ravel(), order)
    assert np.array_equal(np.sort(d), np.arange(n * n))
    inv = np.empty((n * n, 2), dtype=np.int64)
    inv[d] = np.stack([x.ravel(), y.ravel()], axis=1)
    steps = np.abs(np.diff(inv, axis=0)).sum(axis=1)
    assert (steps == 1).all()
    assert inv[0].tolist() == [0, 0] and inv[-1].tolist() == [n - 1, 0]


def test_hilbert_refines_consistently():
    # the order-16 index of a point, divided by 4^(16-k), is the order-k index
    # of its parent cell
    rng = np.random.Generator(np.random.PCG64(11))
    x = rng.integers(0, 1 << 16, 2000)
    y = rng.integers(0, 1 << 16, 2000)
    d16 = om.hilbert_index(x, y, 16)
    for k in (1, 4, 9):
        dk = om.hilbert_index(x >> (16 - k), y >> (16 - k), k)
        np.testing.assert_array_equal(d16 >> (2 * (16 - k)), dk)


def test_sfc_permutation():
    mesh = wl.mesh_c5(n=64, block=8)
    new_of_old, old_of_new = om.sfc_permutation(mesh)
    n = mesh.n_cells
    assert np.array_equal(np.sort(new_of_old), np.arange(n))
    assert np.array_equal(new_of_old[old_of_new], np.arange(n))
    tri = mesh.cell_nodes[old_of_new, 3] < 0
    nq = int((~tri).sum())
    assert not tri[:nq].any() and tri[nq:].all()
    d = om.sfc_keys(mesh)[old_of_new]
    assert (np.diff(d[:nq]) >= 0).all() and (np.diff(d[nq:]) >= 0).all()
