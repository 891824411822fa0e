"""The patch form of the oracle (used at sizes the whole-mesh oracle cannot
reach) equals the whole-mesh oracle at the sampled cells: bit for bit after
an RK3 step, to rounding for the residual."""
import numpy as np
import pytest

import workloads as wl
from oracle import weights as ow
from oracle import scheme as osc
import oracle_patch as op


@pytest.mark.parametrize("name", ["mixed", "sod"])
def test_patch_oracle_equals_whole_mesh_oracle(name):
    if name == "mixed":
        mesh = wl.mesh_c5(n=48, block=12, jitter=0.3, seed=3)
        W = wl.initial_state("c5", mesh, q=2)
    else:
        mesh = wl.mesh_c3(n=40, jitter=0.15, seed=4, band=0.08)
        W = wl.initial_state("c3", mesh)
    ph = osc.Physics("euler")
    T = ow.precompute(mesh)
    dt = 0.5 * osc.cfl_dt(T, W, ph, 0.5)
    ref = osc.rk3_step(T, W, ph, dt)
    L = osc.residual_vectorized(T, W, ph)
    rng = np.random.default_rng(7)
    samples = rng.choice(mesh.n_cells, 5, replace=False)
    if name == "sod":   # a cell on the open boundary and one on the jump
        x = mesh.node_xy[np.maximum(mesh.cell_nodes, 0)].mean(1)
        samples = np.append(samples, [int(np.argmin(x[:, 0])), int(np.argmin(np.abs(
            (x[:, 0] - 0.5) * np.cos(np.pi / 6) + (x[:, 1] - 0.5) * np.sin(np.pi / 6))))])
    inc = op.NodeIncidence(mesh)
    got = op.rk3_at(mesh, W, samples, ph, dt, inc=inc)
    assert np.array_equal(got, ref[:, samples])
    gl = op.residual_at(mesh, W, samples, ph, inc=inc)
    assert np.abs(gl - L[:, samples]).max() <= 1e-12 * np.abs(L).max()


def test_patch_is_local():
    """Too few rings would change the answer: the ring count is tight enough
    to matter, so the test above is not vacuous."""
    mesh = wl.mesh_c5(n=48, block=12, jitter=0.3, seed=3)
    W = wl.seeded_state(mesh, 4, 5)
    ph = osc.Physics("euler")
    T = ow.precompute(mesh)
    ref = osc.rk3_step(T, W, ph, 2e-3)
    inc = op.NodeIncidence(mesh)
    c = 1000
    sub, cells = op.patch_mesh(mesh, inc, c, 2)
    Ts = ow.precompute(sub)
    with np.errstate(invalid="ignore"):
        Ws = osc.rk3_step(Ts, W[:, cells].copy(), ph, 2e-3)
    assert not np.array_equal(Ws[:, np.searchsorted(cells, c)], ref[:, c])
