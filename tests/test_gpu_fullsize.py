"""Parity at the full sizes of the workloads, in the launch shapes the
benchmark uses: one RK3 step of fixed dt on the whole mesh on the GPU,
compared at a few hundred sampled cells (random ones, cells next to a
tile edge of the launch, next to the other cell type, at periodic seams,
open boundaries and the shock) with the oracle evaluated on each sample's
domain of dependence (tests/oracle_patch.py).  Bars, over the samples, both
as relative L1 and element by element against the largest value of each
variable: FP64 <= 1e-12, FP32 (FP64 state) <= 1e-5; results do not depend
on the launch shape (bitwise)."""
import numpy as np
import pytest

import workloads as wl
from oracle import scheme as osc
import oracle_patch as op
from gpu_helpers import physics_for, parity_err

pytestmark = pytest.mark.gpu


def _gpu_step(uw, M, W, precision, dt, schedule="tune"):
    import torch
    ph = physics_for(uw, "euler", precision)
    if schedule == "tune":
        M.autotune(ph)
    else:
        M.schedule(schedule)
    Wd = torch.from_numpy(M.to_internal(W)).to("cuda:0")
    t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    M.rk3_step(ph, Wd, t, dt_fixed=dt)
    M.check()
    return M.to_original(Wd.cpu().numpy())


def _cell_centres(mesh):
    cn = mesh.cell_nodes
    nf = np.where(cn[:, 3] < 0, 3, 4)
    xy = mesh.node_xy[np.maximum(cn, 0)]
    xy = np.where((cn >= 0)[:, :, None], xy, 0.0).sum(1)
    return xy / nf[:, None]


def _edge_classes(mesh, tile=512):
    """Cells whose stencil work crosses a seam of the launch: those with a
    face neighbour in another tile of the internal order (tiles of ``tile``
    consecutive cells of one type; their edges are edges of every smaller
    power-of-two tile as well) and those with a face neighbour of the other
    cell type.  Computed with the oracle's connectivity and its Hilbert
    order (pinned bit-exact against the library's), not the library's."""
    from oracle import mesh as om
    conn = om.connectivity(mesh)
    new_of_old, _ = om.sfc_permutation(mesh)
    is_tri = mesh.cell_nodes[:, 3] < 0
    nq = int((~is_tri).sum())
    pos = new_of_old.astype(np.int64)
    tile_of = np.where(pos < nq, pos // tile, (nq + tile - 1) // tile + (pos - nq) // tile)
    nb = conn.nbr
    has = nb >= 0
    nbc = np.where(has, nb, 0)
    cross_tile = (has & (tile_of[nbc] != tile_of[:, None])).any(1)
    cross_type = (has & (is_tri[nbc] != is_tri[:, None])).any(1)
    return np.flatnonzero(cross_tile), np.flatnonzero(cross_type)


def _pick(rng, pool, k):
    pool = np.asarray(pool)
    return rng.choice(pool, min(k, pool.size), replace=False) if pool.size else pool


def _check(uw, mesh, W, samples, dt, schedules=("tune",)):
    M = uw.Mesh.from_workload(mesh, device=0)
    M.precompute()
    ref = op.rk3_at(mesh, W, samples, osc.Physics("euler"), dt)
    got64 = _gpu_step(uw, M, W, "fp64", dt)
    e64 = parity_err(got64[:, samples], ref, 1e-12)
    got32 = _gpu_step(uw, M, W, "fp32", dt)
    e32 = parity_err(got32[:, samples], ref, 1e-5)
    print(f"{mesh.name}: {mesh.n_cells} cells, {len(samples)} samples, "
          f"fp64 rel err {e64:.3e}, fp32 rel err {e32:.3e}", flush=True)
    assert e64 <= 1e-12
    assert e32 <= 1e-5
    for sch in schedules[1:]:
        again = _gpu_step(uw, M, W, "fp32", dt, sch)
        assert np.array_equal(again, got32), sch
    # the step moved the state: the comparison is not of unchanged values
    assert np.abs(ref - W[:, samples]).max() > 1e-6


@pytest.mark.parametrize("kind", ["quad", "tri"])
def test_density_wave_160k(kind):
    import paper_1712_08317_amd as uw
    mesh = wl.mesh_c2q() if kind == "quad" else wl.mesh_c2t()
    W = wl.initial_state("c2q", mesh)
    rng = np.random.default_rng(21)
    tile_edge, _ = _edge_classes(mesh)
    samples = np.unique(np.concatenate([rng.choice(mesh.n_cells, 100, replace=False),
                                        _pick(rng, tile_edge, 100)]))
    _check(uw, mesh, W, samples, dt=0.1 * mesh.h,
           schedules=("tune", (0, 0, 0), (512, 1024, 2048)))


def test_rotated_sod_2m():
    import paper_1712_08317_amd as uw
    mesh = wl.mesh_c3()
    W = wl.initial_state("c3", mesh)
    c = _cell_centres(mesh)
    rng = np.random.default_rng(22)
    d = (c[:, 0] - 0.5) * np.cos(np.pi / 6) + (c[:, 1] - 0.5) * np.sin(np.pi / 6)
    near = np.flatnonzero(np.abs(d) < 2 * mesh.h)
    edge = np.flatnonzero((c.min(1) < mesh.h) | (c.max(1) > 1 - mesh.h))
    corner = [int(np.argmin(c.sum(1))), int(np.argmax(c.sum(1))),
              int(np.argmin(c[:, 0] - c[:, 1])), int(np.argmax(c[:, 0] - c[:, 1]))]
    tile_edge, interface = _edge_classes(mesh)
    # where the shock band's triangles meet the open boundary
    band_edge = np.intersect1d(np.intersect1d(interface, edge), np.flatnonzero(np.abs(d) < 0.1))
    samples = np.unique(np.concatenate([rng.choice(mesh.n_cells, 50, replace=False),
                                        _pick(rng, near, 40), _pick(rng, edge, 30),
                                        _pick(rng, tile_edge, 40), _pick(rng, interface, 40),
                                        _pick(rng, band_edge, 10), corner]))
    # the fastest signal in the tube moves about 2 length units per time
    _check(uw, mesh, W, samples, dt=0.4 * mesh.h / 2.5)


def test_mixed_vortex_16m():
    import paper_1712_08317_amd as uw
    mesh = wl.mesh_c5()
    W = wl.initial_state("c5", mesh)
    c = _cell_centres(mesh)
    rng = np.random.default_rng(23)
    core = np.flatnonzero(np.hypot(c[:, 0] - 1, c[:, 1] - 1) < 0.2)
    seam = np.flatnonzero((c.min(1) < mesh.h) | (c.max(1) > 2 - mesh.h))
    tile_edge, interface = _edge_classes(mesh)
    samples = np.unique(np.concatenate([rng.choice(mesh.n_cells, 50, replace=False),
                                        _pick(rng, core, 40), _pick(rng, seam, 30),
                                        _pick(rng, tile_edge, 50), _pick(rng, interface, 50),
                                        _pick(rng, np.intersect1d(seam, interface), 20)]))
    _check(uw, mesh, W, samples, dt=0.3 * mesh.h / 3.0)


def test_batch_256_instances():
    import torch
    import paper_1712_08317_amd as uw
    meshes = [wl.mesh_c4(k) for k in range(256)]
    Ms = [uw.Mesh.from_workload(m, device=0) for m in meshes]
    for M in Ms:
        M.precompute()
    states = [wl.initial_state("c2q", m, q=2) for m in meshes]
    dt = 4e-4
    rng = np.random.default_rng(24)
    pick = rng.choice(256, 32, replace=False)
    refs = {}
    for k in pick:
        # the first and last cells of an instance sit next to the
        # neighbouring instances in the concatenated state
        n = meshes[k].n_cells
        samples = np.unique(np.concatenate([rng.choice(n, 4, replace=False), [0, n - 1]]))
        refs[int(k)] = (samples, op.rk3_at(meshes[k], states[k], samples,
                                           osc.Physics("euler"), dt))
    out, long = {}, {}
    for prec in ("fp64", "fp32"):
        ph = physics_for(uw, "euler", prec)
        B = uw.Batch(Ms, ph)
        B.autotune(ph)
        Wb = torch.from_numpy(B.to_internal(states)).to("cuda:0")
        tb = torch.zeros(256, dtype=torch.float64, device="cuda:0")
        B.rk3_step(Wb, tb, dt_fixed=dt, n_steps=1)
        B.check()
        out[prec] = B.to_original(Wb.cpu().numpy())
        # the workload as specified: 100 RK3 steps of every instance, each
        # with its own CFL time step, as captured graph replays
        Wb = torch.from_numpy(B.to_internal(states)).to("cuda:0")
        tb.zero_()
        for _ in range(10):
            B.rk3_step(Wb, tb, cfl=0.5, n_steps=10)
        B.check()
        long[prec] = (B.to_original(Wb.cpu().numpy()), tb.cpu().numpy())
        print(f"{prec}: tile {B.tile_size()}, schedule {B.schedule()}, 100 steps to "
              f"t in [{tb.min().item():.4f}, {tb.max().item():.4f}]", flush=True)
        del Wb, B
    got = {p: np.concatenate([out[p][k][:, refs[k][0]] for k in refs], 1) for p in out}
    ref = np.concatenate([refs[k][1] for k in refs], 1)
    e64, e32 = parity_err(got["fp64"], ref, 1e-12), parity_err(got["fp32"], ref, 1e-5)
    print(f"batch of 256 ({sum(m.n_cells for m in meshes)} cells): fp64 {e64:.3e}, "
          f"fp32 {e32:.3e}", flush=True)
    assert e64 <= 1e-12
    assert e32 <= 1e-5
    # FP32 against FP64 on the same device after 100 steps, every instance
    worst = max(parity_err(a, b, 1e-5) for a, b in zip(long["fp32"][0], long["fp64"][0]))
    print(f"100 steps, fp32 vs fp64, worst instance: {worst:.3e}", flush=True)
    assert worst <= 1e-5
    # the CFL steps depend on the state: FP32 and FP64 times agree closely
    assert np.allclose(long["fp32"][1], long["fp64"][1], rtol=1e-6, atol=0)


def test_rotated_sod_fp32_long_run():
    """FP32 arithmetic against FP64 on the same device over 300 steps of the
    2M-cell shock tube: every conserved variable within 1e-5 relative L1.
    The momentum components are zero outside the waves, so this needs the
    resting gas to stay at rest in FP32 (exact zero-velocity face fluxes and
    FP64 closure of the gather); an FP64 run from a start perturbed at FP32
    rounding level is printed beside it for scale."""
    import torch
    import paper_1712_08317_amd as uw
    mesh = wl.mesh_c3()
    W0 = wl.initial_state("c3", mesh)
    M = uw.Mesh.from_workload(mesh, device=0)
    M.precompute()
    # CFL about 0.55 in the triangle band (half-size cells), 0.3 elsewhere
    dt = 0.2 * mesh.h / 2.5

    def run(prec, W, steps=300):
        ph = physics_for(uw, "euler", prec)
        Wd = torch.from_numpy(M.to_internal(W)).to("cuda:0")
        t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        for _ in range(steps):
            M.rk3_step(ph, Wd, t, dt_fixed=dt)
        M.check()
        return M.to_original(Wd.cpu().numpy())

    a, b = run("fp32", W0), run("fp64", W0)
    rng = np.random.default_rng(3)
    p = run("fp64", W0 * (1 + 6e-8 * rng.uniform(-1, 1, W0.shape)))
    num, den = np.abs(a - b).sum(1), np.abs(b).sum(1)
    per = num / den
    ctl = np.abs(p - b).sum(1) / den
    print(f"per variable {per}, state {num.sum() / den.sum():.3e}, perturbed fp64 {ctl}",
          flush=True)
    assert (per <= 1e-5).all()
