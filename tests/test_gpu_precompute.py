"""The FP64 precompute on the GPU against the same routine on host threads
and against the oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle import weights as ow

pytestmark = pytest.mark.gpu

MESHES = {
    "mixed": lambda: wl.mesh_c5(n=32, block=8, jitter=0.3, seed=61),
    "sod": lambda: wl.mesh_c3(n=30, jitter=0.15, seed=62, band=0.1),
    "tri30": lambda: wl.grid_mesh(14, 14, 2.0, 2.0, "tri", 0.3, 63, True),
}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("d_scope", [0, 1])
def test_device_precompute_matches_host(name, d_scope):
    import paper_1712_08317_amd as uw
    mesh = MESHES[name]()
    Md = uw.Mesh.from_workload(mesh, device=0)
    Mh = uw.Mesh.from_workload(mesh, device=-1)
    sc = uw.make_scheme(d_scope=d_scope, mode=uw.UW_WENO)
    dd = Md.precompute(sc)
    dh = Mh.precompute(sc)
    assert dd["n_absent_slots"] == dh["n_absent_slots"]
    assert dd["n_rank_deficient"] == dh["n_rank_deficient"]
    assert abs(dd["max_abs_gamma_opt"] / dh["max_abs_gamma_opt"] - 1) < 1e-9
    for which in range(6):
        a, b = Md.table(which), Mh.table(which)
        scale = max(1.0, np.abs(b).max())
        assert np.abs(a - b).max() <= 1e-10 * scale, which


def test_device_precompute_matches_oracle():
    import paper_1712_08317_amd as uw
    mesh = MESHES["mixed"]()
    M = uw.Mesh.from_workload(mesh, device=0)
    M.precompute()
    T = ow.precompute(mesh)
    gam = M.table(0)
    for nf, g in T.groups.items():
        rows = M.new_of_old[g.st.cells]
        G, Mc = 2 * nf, g.st.spec.M
        assert np.abs(gam[rows][:, :G, :Mc] - g.gamma).max() < 1e-10 * max(1, np.abs(g.gamma).max())
