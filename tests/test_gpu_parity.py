"""Parity of the HIP path with the oracle (element by element, same seeded
inputs).  Bars: FP64 relative L1 <= 1e-12, FP32 (FP64 state) <= 1e-5."""
import numpy as np
import pytest

import workloads as wl
from oracle import weights as ow
from oracle import scheme as osc
from gpu_helpers import rel_l1, gpu_residual, physics_for, small_meshes, parity_err

pytestmark = pytest.mark.gpu

MESHES = small_meshes()
_cache = {}


def _setup(name, mode="weno"):
    key = (name, mode)
    if key not in _cache:
        import paper_1712_08317_amd as uw
        mesh = MESHES[name]
        M = uw.Mesh.from_workload(mesh, device=0)
        M.precompute(uw.make_scheme(mode=uw.UW_LINEAR if mode == "linear" else uw.UW_WENO))
        T = ow.precompute(mesh, ow.Scheme(mode=mode))
        _cache[key] = (uw, mesh, M, T)
    return _cache[key]


def _state(name, mesh, seed, mode="weno"):
    if name == "c1":
        return wl.seeded_state(mesh, 1, seed)
    if name == "sod" and mode == "weno":
        # the unlimited linear scheme gives negative pressure at the shock
        # tube's jump, so the linear mode is compared on a smooth state
        return wl.initial_state("c3", mesh)
    return wl.seeded_state(mesh, 4, seed)


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("mode", ["weno", "linear"])
def test_residual_fp64(name, mode):
    uw, mesh, M, T = _setup(name, mode)
    eq = "advection" if name == "c1" else "euler"
    W = _state(name, mesh, 11, mode)
    ref = osc.residual_vectorized(T, W, osc.Physics(eq))
    assert np.isfinite(ref).all()
    got = gpu_residual(uw, M, W, eq, "fp64")
    print(name, mode, "rel L1 / elementwise", parity_err(got, ref, 1e-12))
    assert parity_err(got, ref, 1e-12) <= 1e-12


@pytest.mark.parametrize("name", list(MESHES))
def test_residual_fp32(name):
    uw, mesh, M, T = _setup(name)
    eq = "advection" if name == "c1" else "euler"
    W = _state(name, mesh, 12)
    ref = osc.residual_vectorized(T, W, osc.Physics(eq))
    got = gpu_residual(uw, M, W, eq, "fp32")
    print(name, "fp32 rel L1", parity_err(got, ref, 1e-5))
    assert parity_err(got, ref, 1e-5) <= 1e-5


def test_uniform_state_and_conservation():
    import torch
    uw, mesh, M, T = _setup("mixed")
    W = np.tile(np.array([[1.3], [0.2], [-0.7], [4.1]]), (1, mesh.n_cells))
    for prec in ("fp64", "fp32"):
        L = gpu_residual(uw, M, W, "euler", prec)
        assert np.abs(L).max() < (1e-11 if prec == "fp64" else 2e-4)
    # gas at rest: every face flux is exactly (0, p n, 0) in either precision,
    # and the FP64 gather with closed face factors cancels it to FP64 rounding
    Wr = np.tile(np.array([[1.3], [0.0], [0.0], [4.1]]), (1, mesh.n_cells))
    for prec in ("fp64", "fp32"):
        L = gpu_residual(uw, M, Wr, "euler", prec)
        assert np.abs(L).max() < 1e-11, prec
    Ws = wl.seeded_state(mesh, 4, 13)
    L = gpu_residual(uw, M, Ws, "euler", "fp64")
    area = np.zeros(mesh.n_cells)
    for g in T.groups.values():
        area[g.st.cells] = g.area
    tot = np.abs((L * area).sum(axis=1))
    assert (tot < 1e-12 * np.abs(L * area).sum(axis=1)).all()
    del torch


def test_bitwise_reproducible():
    import torch
    uw, mesh, M, T = _setup("mixed")
    W = _state("mixed", mesh, 14)
    for prec in ("fp64", "fp32"):
        a = gpu_residual(uw, M, W, "euler", prec)
        b = gpu_residual(uw, M, W, "euler", prec)
        assert np.array_equal(a, b)
    del torch


@pytest.mark.parametrize("name", ["c1", "mixed", "sod"])
def test_rk3_steps_fp64_match_oracle(name):
    import torch
    uw, mesh, M, T = _setup(name)
    eq = "advection" if name == "c1" else "euler"
    W = wl.initial_state("c1", mesh) if name == "c1" else _state(name, mesh, 15)
    ph = osc.Physics(eq)
    dt = 0.5 * osc.cfl_dt(T, W, ph, 0.5)
    ref = W.copy()
    for _ in range(3):
        ref = osc.rk3_step(T, ref, ph, dt)
    Wd = torch.from_numpy(M.to_internal(W)).to("cuda:0")
    t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    for _ in range(3):
        M.rk3_step(physics_for(uw, eq, "fp64"), Wd, t, dt_fixed=dt)
    M.check()
    got = M.to_original(Wd.cpu().numpy())
    print(name, "rk3 rel L1", parity_err(got, ref, 1e-12))
    assert parity_err(got, ref, 1e-12) <= 1e-12
    assert abs(t.item() - 3 * dt) <= 1e-15


def test_c1_to_final_time_with_device_cfl():
    """Configuration 1: scalar advection, FP64, CFL 0.5 to t = 0.2 with the
    time step chosen on the device; the oracle repeats the same steps."""
    import torch
    uw, mesh, M, T = _setup("c1")
    W0 = wl.initial_state("c1", mesh)
    ph = osc.Physics("advection")
    Wd = torch.from_numpy(M.to_internal(W0)).to("cuda:0")
    t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    ref = W0.copy()
    tr = 0.0
    steps = 0
    while tr < 0.2 - 1e-14 and steps < 100:
        dt = min(osc.cfl_dt(T, ref, ph, 0.5), 0.2 - tr)
        ref = osc.rk3_step(T, ref, ph, dt)
        tr += dt
        M.rk3_step(physics_for(uw, "advection", "fp64"), Wd, t, cfl=0.5, t_end=0.2)
        steps += 1
    torch.cuda.synchronize()
    assert abs(t.item() - 0.2) < 1e-13
    got = M.to_original(Wd.cpu().numpy())
    assert parity_err(got, ref, 1e-12) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cfl_dt_matches_oracle(prec):
    import torch
    uw, mesh, M, T = _setup("mixed")
    W = wl.seeded_state(mesh, 4, 16)
    ref = osc.cfl_dt(T, W, osc.Physics("euler"), 0.5)
    Wd = torch.from_numpy(M.to_internal(W)).to("cuda:0")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    M.cfl_dt(physics_for(uw, "euler", prec), Wd, 0.5, dt)
    torch.cuda.synchronize()
    assert abs(dt.item() / ref - 1) < (1e-13 if prec == "fp64" else 1e-6)


def test_fp32_solution_within_1e5_of_fp64_oracle():
    """FP32 arithmetic with FP64 state: after 10 steps of the smooth mixed-mesh
    Euler problem the relative L1 error against the FP64 oracle is <= 1e-5."""
    import torch
    uw, mesh, M, T = _setup("mixed")
    W0 = wl.initial_state("c5", mesh)
    ph = osc.Physics("euler")
    dt = osc.cfl_dt(T, W0, ph, 0.5)
    ref = W0.copy()
    for _ in range(10):
        ref = osc.rk3_step(T, ref, ph, dt)
    Wd = torch.from_numpy(M.to_internal(W0)).to("cuda:0")
    t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    for _ in range(10):
        M.rk3_step(physics_for(uw, "euler", "fp32"), Wd, t, dt_fixed=dt)
    M.check()
    got = M.to_original(Wd.cpu().numpy())
    err = parity_err(got, ref, 1e-5)
    print("fp32 10-step rel L1", err)
    assert err <= 1e-5


def test_nonfinite_state_is_flagged():
    import torch
    uw, mesh, M, T = _setup("quad")
    W = wl.seeded_state(mesh, 4, 17)
    W[0, 5] = np.nan
    Wd = torch.from_numpy(M.to_internal(W)).to("cuda:0")
    t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    M.rk3_step(physics_for(uw, "euler", "fp64"), Wd, t, dt_fixed=1e-3)
    with pytest.raises(uw.UwError) as e:
        M.check()
    assert e.value.status == uw.UW_ENONFINITE
    M.check()   # the flag was cleared


# ---------------------------------------------------------------------------
# WENO on the characteristic variables (Sec. 4, Euler)
# ---------------------------------------------------------------------------

_char_cache = {}


def _setup_char(name):
    if name not in _char_cache:
        import paper_1712_08317_amd as uw
        mesh = MESHES[name]
        M = uw.Mesh.from_workload(mesh, device=0)
        M.precompute(uw.make_scheme(variables=uw.UW_CHARACTERISTIC))
        T = ow.precompute(mesh, ow.Scheme(variables="characteristic"))
        _char_cache[name] = (uw, mesh, M, T)
    return _char_cache[name]


@pytest.mark.parametrize("name", ["quad", "tri", "mixed", "sod"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_characteristic_residual_matches_oracle(name, prec):
    uw, mesh, M, T = _setup_char(name)
    W = wl.initial_state("c3", mesh) if name == "sod" else wl.seeded_state(mesh, 4, 15)
    ref = osc.residual_vectorized(T, W, osc.Physics("euler"))
    got = gpu_residual(uw, M, W, "euler", prec)
    tol = 1e-12 if prec == "fp64" else 1e-5
    err = parity_err(got, ref, tol)
    print(name, prec, "characteristic rel L1", err)
    assert err <= tol
    # the characteristic reconstruction is not the conserved one
    if prec == "fp64":
        T0 = ow.precompute(mesh)
        assert rel_l1(osc.residual_vectorized(T0, W, osc.Physics("euler")), ref) > 1e-6


def test_characteristic_rk3_steps_match_oracle():
    import torch
    uw, mesh, M, T = _setup_char("sod")
    W = wl.initial_state("c3", mesh)
    ph = osc.Physics("euler")
    dt = 0.3 * osc.cfl_dt(T, W, ph, 1.0)
    ref = W
    for _ in range(3):
        ref = osc.rk3_step(T, ref, ph, dt)
    Wd = torch.from_numpy(M.to_internal(W)).to("cuda:0")
    t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    p64 = physics_for(uw, "euler", "fp64")
    for _ in range(3):
        M.rk3_step(p64, Wd, t, dt_fixed=dt)
    M.check()
    got = M.to_original(Wd.cpu().numpy())
    print("characteristic sod rk3 rel L1", parity_err(got, ref, 1e-12))
    assert parity_err(got, ref, 1e-12) <= 1e-12


def test_single_mesh_graph_replays_match_eager_steps():
    """uw_rk3_step replays a captured graph when per-kernel timing is off and
    launches eagerly when it is on: the two give the same bits, replay after
    replay, with unrelated device work in between."""
    import torch
    uw, mesh, M, T = _setup("mixed")
    W = wl.seeded_state(mesh, 4, 16)
    for prec in ("fp64", "fp32"):
        ph = physics_for(uw, "euler", prec)
        Wg = torch.from_numpy(M.to_internal(W)).to("cuda:0")
        We = Wg.clone()
        tg = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        te = tg.clone()
        for rep in range(3):
            M.profile(enable=0)
            M.rk3_step(ph, Wg, tg, cfl=0.4)
            noise = torch.randn(1000, device="cuda:0").sum()
            torch.cuda.synchronize()
            del noise
            M.profile(enable=1)
            M.rk3_step(ph, We, te, cfl=0.4)
            M.profile(enable=0)
            torch.cuda.synchronize()
            assert torch.equal(Wg, We), (prec, rep)
            assert tg.item() == te.item()
        M.check()


def test_graphs_follow_physics_and_moved_work_buffers():
    """A captured step is tied to its physics (gamma, advection velocity)
    and to the library's work buffers: a call with other physics on the
    same state captures anew, and a call that needs larger buffers (Euler
    after scalar advection) retires the graphs that held the old ones.
    Each graph result is checked against eager launches."""
    import torch
    import paper_1712_08317_amd as uw
    mesh = wl.grid_mesh(16, 16, 2.0, 2.0, "tri", 0.2, 21, True)

    def run(graph, seq):
        M = uw.Mesh.from_workload(mesh, device=0)
        M.precompute()
        M.profile(enable=0 if graph else 1)
        Wa = torch.from_numpy(M.to_internal(wl.seeded_state(mesh, 1, 22))).to("cuda:0")
        We = torch.from_numpy(M.to_internal(wl.seeded_state(mesh, 4, 23))).to("cuda:0")
        ta = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        te = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        for what, gamma, ax in seq:
            if what == "adv":
                M.rk3_step(uw.make_physics(uw.UW_ADVECTION, ax, 1.0, 1.4, uw.UW_FP64), Wa, ta,
                           dt_fixed=0.01)
            else:
                M.rk3_step(uw.make_physics(uw.UW_EULER, 1.0, 1.0, gamma, uw.UW_FP64), We, te,
                           dt_fixed=0.005)
        torch.cuda.synchronize()
        M.check()
        return Wa.cpu(), We.cpu()

    seq = [("adv", 1.4, 1.0), ("euler", 1.4, 1.0), ("adv", 1.4, 1.0), ("adv", 1.4, -0.5),
           ("euler", 1.67, 1.0), ("euler", 1.4, 1.0)]
    ga, ge = run(True, seq)
    ea, ee = run(False, seq)
    assert torch.equal(ga, ea) and torch.equal(ge, ee)


@pytest.mark.parametrize("name", ["mixed", "quad", "tri", "sod"])
def test_tile_sizes_fp32_match_oracle(name):
    """The stage kernels with 512-cell tiles (FP32, WENO on the conserved
    variables): a residual and three RK3 steps against the oracle, and the
    kernels that exist for 256-cell tiles only refuse the tile size."""
    import torch
    uw, mesh, M, T = _setup(name)
    W = _state(name, mesh, 16)
    try:
        assert M.tile_size(512) == 512
        ref = osc.residual_vectorized(T, W, osc.Physics("euler"))
        got = gpu_residual(uw, M, W, "euler", "fp32")
        assert parity_err(got, ref, 1e-5) <= 1e-5
        with pytest.raises(uw.UwError) as e:
            gpu_residual(uw, M, W, "euler", "fp64")
        assert e.value.status == uw.UW_EINVAL
        ph = osc.Physics("euler")
        dt = 0.5 * osc.cfl_dt(T, W, ph, 0.5)
        ref = W.copy()
        for _ in range(3):
            ref = osc.rk3_step(T, ref, ph, dt)
        Wd = torch.from_numpy(M.to_internal(W)).to("cuda:0")
        t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        for _ in range(3):
            M.rk3_step(physics_for(uw, "euler", "fp32"), Wd, t, dt_fixed=dt)
        M.check()
        err = parity_err(M.to_original(Wd.cpu().numpy()), ref, 1e-5)
        print(name, "tile 512 fp32 rk3 rel err", err)
        assert err <= 1e-5
    finally:
        M.tile_size(256)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_step_call_equals_single_steps(prec):
    """uw_rk3_steps: the last stage of each step forms the next step's CFL
    bound; the states and times equal those of single-step calls, which
    form it in a pass of their own, bit for bit (graph replay and eager
    launches alike)."""
    import torch
    uw, mesh, M, T = _setup("mixed")
    W = _state("mixed", mesh, 17)
    ph = physics_for(uw, "euler", prec)
    runs = {}
    for how in ("single", "multi", "multi-eager"):
        Wd = torch.from_numpy(M.to_internal(W)).to("cuda:0")
        t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        M.profile(enable=1 if how == "multi-eager" else 0)
        if how == "single":
            for _ in range(4):
                M.rk3_step(ph, Wd, t, cfl=0.5)
        else:
            M.rk3_steps(ph, Wd, t, 4, cfl=0.5)
        M.profile(enable=0)
        M.check()
        runs[how] = (Wd.cpu().numpy(), t.item())
    ref = runs["single"]
    for how in ("multi", "multi-eager"):
        assert np.array_equal(runs[how][0], ref[0]), how
        assert runs[how][1] == ref[1], how
    assert ref[1] > 0.0


def test_graph_cache_keeps_a_bounded_number_of_graphs():
    """Captured steps are keyed by their arguments; a caller that changes
    the fixed step every call gets correct results from an evicting cache
    (at most 8 graphs), equal to eager launches."""
    import torch
    uw, mesh, M, T = _setup("tri")
    W = _state("tri", mesh, 18)
    ph = physics_for(uw, "euler", "fp64")
    runs = {}
    for graph in (True, False):
        Wd = torch.from_numpy(M.to_internal(W)).to("cuda:0")
        t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        M.profile(enable=0 if graph else 1)
        for k in range(20):
            M.rk3_step(ph, Wd, t, dt_fixed=1e-4 * (1 + (k % 11)))
        M.profile(enable=0)
        M.check()
        runs[graph] = (Wd.cpu().numpy(), t.item())
    assert np.array_equal(runs[True][0], runs[False][0])
    assert runs[True][1] == runs[False][1]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("scheme,tile", [("weno", 256), ("weno", 512), ("linear", 256),
                                         ("characteristic", 256)])
def test_one_reconstruction_launch_for_both_cell_types(prec, scheme, tile):
    """Schedule (q, -1, f): both cell types reconstructed by one launch (any
    number of persistent blocks, each taking quadrilateral and triangle
    tiles) give the residual of the separate launches bit for bit, for the
    Euler equations and scalar advection; the FP32 linear scheme, whose two
    kernels differ in occupancy, keeps separate launches."""
    if tile == 512 and (prec != "fp32" or scheme != "weno"):
        pytest.skip("512-cell tiles: FP32 WENO on the conserved variables only")
    import paper_1712_08317_amd as uw
    for name in ("mixed", "sod"):
        mesh = MESHES[name]
        M = uw.Mesh.from_workload(mesh, device=0)
        M.precompute(uw.make_scheme(
            mode=uw.UW_LINEAR if scheme == "linear" else uw.UW_WENO,
            variables=uw.UW_CHARACTERISTIC if scheme == "characteristic" else uw.UW_CONSERVED))
        if tile != 256:
            assert M.tile_size(tile) == tile
        W = wl.seeded_state(mesh, 4, 23) if not (name == "sod" and scheme == "linear") \
            else wl.initial_state("c3", mesh)
        equations = ["euler"] + (["advection"] if scheme != "characteristic" else [])
        for eq in equations:
            Wq = W if eq == "euler" else W[:1].copy()
            M.schedule((0, 0, 0))
            ref = gpu_residual(uw, M, Wq, eq, prec)
            for q in (0, 2, 256):
                assert M.schedule((q, -1, 0)) == (q, -1, 0)
                got = gpu_residual(uw, M, Wq, eq, prec)
                assert np.array_equal(got, ref), (name, eq, q)
        with pytest.raises(uw.UwError) as e:
            M.schedule((0, -2, 0))
        assert e.value.status == uw.UW_EINVAL
