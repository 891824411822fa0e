"""Python binding of the uweno C-ABI (include/uweno.h).

Argument marshalling only: every step of the per-stage operator runs in the
HIP kernels of ``libuweno.so``.  PyTorch supplies device memory and streams.
The library must have been built (``python paper_1712_08317_amd/build.py``);
importing this module raises if it is missing.

Typical use (state ``W`` as cell averages [V, n] in the mesh's own order)::

    import torch, paper_1712_08317_amd as uw
    M = uw.Mesh(node_xy, cell_nodes, bc=uw.UW_BC_TRANSMISSIVE)   # renumbered
    M.precompute(uw.make_scheme(variables=uw.UW_CHARACTERISTIC))
    ph = uw.make_physics(uw.UW_EULER, precision=uw.UW_FP32)
    Wd = torch.from_numpy(M.to_internal(W)).cuda()
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        M.rk3_step(ph, Wd, t, cfl=0.5, t_end=t_end)
    M.check()                                   # raises on NaN or rho, p <= 0
    W = M.to_original(Wd.cpu().numpy())
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# UWENO_LIB may name another build of the library (default: the in-tree one)
LIB_PATH = os.environ.get("UWENO_LIB", os.path.join(HERE, "libuweno.so"))

UW_OK, UW_EINVAL, UW_EMESH, UW_ESTATE, UW_ENOMEM, UW_EDEVICE, UW_ENONFINITE = range(7)
UW_BC_PERIODIC, UW_BC_TRANSMISSIVE, UW_BC_REFLECTIVE, UW_BC_INFLOW = 0, 1, 2, 3
UW_BC_FRONT = 1 << 16
UW_WENO, UW_LINEAR = 0, 1
UW_CONSERVED, UW_CHARACTERISTIC = 0, 1
UW_D_PER_GP, UW_D_PER_CELL = 0, 1
UW_ADVECTION, UW_EULER = 0, 1
UW_FP64, UW_FP32 = 0, 1

STATUS_NAMES = {0: "UW_OK", 1: "UW_EINVAL", 2: "UW_EMESH", 3: "UW_ESTATE", 4: "UW_ENOMEM",
                5: "UW_EDEVICE", 6: "UW_ENONFINITE"}


class UwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("node_xy", ctypes.c_void_p),
                ("n_cells", ctypes.c_int64), ("cell_nodes", ctypes.c_void_p),
                ("node_id", ctypes.c_void_p), ("bc", ctypes.c_int32),
                ("face_bc", ctypes.c_void_p), ("n_inflow", ctypes.c_int32),
                ("inflow_W", ctypes.c_void_p), ("n_fronts", ctypes.c_int32),
                ("fronts", ctypes.c_void_p)]


class SchemeC(ctypes.Structure):
    _fields_ = [("zeta", ctypes.c_double), ("theta", ctypes.c_double), ("eps", ctypes.c_double),
                ("optimize", ctypes.c_int32), ("d_scope", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("variables", ctypes.c_int32)]


class PhysicsC(ctypes.Structure):
    _fields_ = [("equation", ctypes.c_int32), ("ax", ctypes.c_double), ("ay", ctypes.c_double),
                ("gamma", ctypes.c_double), ("precision", ctypes.c_int32)]


class DiagC(ctypes.Structure):
    _fields_ = [("max_abs_gamma_raw", ctypes.c_double), ("max_abs_gamma_opt", ctypes.c_double),
                ("resid_opt", ctypes.c_double), ("sum_dev", ctypes.c_double),
                ("n_absent_slots", ctypes.c_int64), ("n_rank_deficient", ctypes.c_int64)]


EXPORTS = ["uw_last_error", "uw_mesh_upload", "uw_mesh_info", "uw_mesh_export",
           "uw_precompute_geometry", "uw_mesh_table", "uw_residual", "uw_residual_at",
           "uw_residual_noalloc", "uw_rk3_step", "uw_rk3_steps",
           "uw_cfl_dt",
           "uw_batch_create", "uw_batch_offsets", "uw_batch_rk3_step", "uw_autotune", "uw_check",
           "uw_profile", "uw_schedule", "uw_tile_size", "uw_mesh_destroy", "uw_batch_destroy"]


def _load():
    # torch ships its own HIP runtime (same soname as /opt/rocm's); loading it
    # first makes this library bind to that one, so both share one runtime
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python paper_1712_08317_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "uw_last_error": (ctypes.c_char_p, []),
        "uw_mesh_upload": (i32, [ctypes.POINTER(MeshDesc), ctypes.c_int, ctypes.POINTER(vp)]),
        "uw_mesh_info": (i32, [vp, vp, vp, vp, vp]),
        "uw_mesh_export": (i32, [vp, vp, vp, vp]),
        "uw_precompute_geometry": (i32, [vp, ctypes.POINTER(SchemeC), ctypes.POINTER(DiagC)]),
        "uw_mesh_table": (i32, [vp, i32, vp]),
        "uw_residual": (i32, [vp, ctypes.POINTER(PhysicsC), vp, vp, vp]),
        "uw_residual_at": (i32, [vp, ctypes.POINTER(PhysicsC), vp, vp, dbl, vp]),
        "uw_residual_noalloc": (i32, [vp, ctypes.POINTER(PhysicsC), vp, vp, vp]),
        "uw_rk3_step": (i32, [vp, ctypes.POINTER(PhysicsC), vp, dbl, dbl, dbl, vp, vp]),
        "uw_rk3_steps": (i32, [vp, ctypes.POINTER(PhysicsC), vp, dbl, dbl, dbl, i32, vp, vp]),
        "uw_cfl_dt": (i32, [vp, ctypes.POINTER(PhysicsC), vp, dbl, vp, vp]),
        "uw_batch_create": (i32, [vp, i32, ctypes.POINTER(PhysicsC), ctypes.POINTER(vp)]),
        "uw_batch_offsets": (i32, [vp, vp]),
        "uw_batch_rk3_step": (i32, [vp, vp, dbl, dbl, dbl, i32, vp, vp]),
        "uw_autotune": (i32, [vp, vp, ctypes.POINTER(PhysicsC), ctypes.c_char_p, vp]),
        "uw_check": (i32, [vp, vp, vp]),
        "uw_profile": (i32, [vp, i32, vp, vp]),
        "uw_schedule": (i32, [vp, vp, vp, vp]),
        "uw_tile_size": (i32, [vp, vp, i32, vp]),
        "uw_mesh_destroy": (None, [vp]),
        "uw_batch_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    del i64
    return lib


LIB = _load()


def _check(status):
    if status != UW_OK:
        raise UwError(status, LIB.uw_last_error().decode())


def _ptr(t):
    """Device or host address of a torch tensor or numpy array."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _device_buffer(x, device, numel, name, at_least=False):
    """Checks a device argument before its address reaches the library,
    which cannot check device pointers: a contiguous FP64 torch tensor on
    the mesh's device holding exactly `numel` values (at least, for
    at_least).  Raises ValueError otherwise."""
    import torch
    if not isinstance(x, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor on cuda:{device}, got {type(x).__name__}")
    if x.dtype != torch.float64:
        raise ValueError(f"{name} must be float64, got {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if (x.numel() < numel) if at_least else (x.numel() != numel):
        want = f"at least {numel}" if at_least else str(numel)
        raise ValueError(f"{name} must hold {want} values, has {x.numel()}")
    if not x.is_cuda or x.device.index != device:
        raise ValueError(f"{name} must be on cuda:{device}, is on {x.device}")


def _nvar(physics):
    """Variables per cell of an equation, or None for an unknown one (the
    library rejects it)."""
    return {UW_EULER: 4, UW_ADVECTION: 1}.get(int(physics.equation))


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def make_scheme(zeta=1e-14, theta=3.0, eps=1e-3, optimize=True, d_scope=UW_D_PER_GP,
                mode=UW_WENO, variables=UW_CONSERVED) -> SchemeC:
    return SchemeC(zeta, theta, eps, int(optimize), d_scope, mode, variables)


def make_physics(equation=UW_EULER, ax=1.0, ay=1.0, gamma=1.4, precision=UW_FP64) -> PhysicsC:
    return PhysicsC(equation, ax, ay, gamma, precision)


class Mesh:
    """A mesh uploaded to the library (internal Hilbert numbering)."""

    def __init__(self, node_xy, cell_nodes, node_id=None, bc=UW_BC_PERIODIC, device=0,
                 face_bc=None, inflow=None, fronts=None):
        self._xy = np.ascontiguousarray(node_xy, dtype=np.float64)
        self._cn = np.ascontiguousarray(cell_nodes, dtype=np.int32)
        self._nid = None if node_id is None else np.ascontiguousarray(node_id, dtype=np.int32)
        self._fbc = None if face_bc is None else np.ascontiguousarray(face_bc, dtype=np.int32)
        self._inf = (None if inflow is None
                     else np.ascontiguousarray(np.asarray(inflow, dtype=np.float64).reshape(-1, 4)))
        self._fr = (None if fronts is None
                    else np.ascontiguousarray(np.asarray(fronts, dtype=np.float64).reshape(-1, 12)))
        desc = MeshDesc(self._xy.shape[0], self._xy.ctypes.data, self._cn.shape[0],
                        self._cn.ctypes.data, None if self._nid is None else self._nid.ctypes.data,
                        bc, None if self._fbc is None else self._fbc.ctypes.data,
                        0 if self._inf is None else self._inf.shape[0],
                        None if self._inf is None else self._inf.ctypes.data,
                        0 if self._fr is None else self._fr.shape[0],
                        None if self._fr is None else self._fr.ctypes.data)
        h = ctypes.c_void_p()
        _check(LIB.uw_mesh_upload(ctypes.byref(desc), device, ctypes.byref(h)))
        self.handle = h
        self.device = device
        n = ctypes.c_int64()
        nq = ctypes.c_int64()
        nfc = ctypes.c_int64()
        self.new_of_old = np.empty(self._cn.shape[0], dtype=np.int32)
        _check(LIB.uw_mesh_info(h, ctypes.byref(n), ctypes.byref(nq), ctypes.byref(nfc),
                                self.new_of_old.ctypes.data))
        self.n_cells, self.n_quads, self.n_interior_faces = n.value, nq.value, nfc.value
        self.old_of_new = np.empty_like(self.new_of_old)
        self.old_of_new[self.new_of_old] = np.arange(self.n_cells, dtype=np.int32)
        self.diag = None

    @classmethod
    def from_workload(cls, mesh, device=0):
        bc = UW_BC_PERIODIC if mesh.bc == "periodic" else UW_BC_TRANSMISSIVE
        return cls(mesh.node_xy, mesh.cell_nodes, mesh.node_id, bc, device,
                   getattr(mesh, "face_bc", None), getattr(mesh, "inflow", None),
                   getattr(mesh, "fronts", None))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and LIB is not None:
            LIB.uw_mesh_destroy(h)
            self.handle = None

    def export(self):
        n = self.n_cells
        slots = np.empty((n, 13), dtype=np.int32)
        present = np.empty((n, 13), dtype=np.uint8)
        nbr = np.empty((n, 4), dtype=np.int32)
        _check(LIB.uw_mesh_export(self.handle, slots.ctypes.data, present.ctypes.data,
                                  nbr.ctypes.data))
        return slots, present, nbr

    def precompute(self, scheme: SchemeC | None = None):
        scheme = scheme or make_scheme()
        d = DiagC()
        _check(LIB.uw_precompute_geometry(self.handle, ctypes.byref(scheme), ctypes.byref(d)))
        self.diag = {name: getattr(d, name) for name, _ in DiagC._fields_}
        return self.diag

    def table(self, which: int):
        shapes = {0: (8, 12), 1: (8, 13), 2: (12, 4), 3: (8, 2), 4: (4, 3), 5: (8, 12)}
        out = np.empty((self.n_cells,) + shapes[which], dtype=np.float64)
        _check(LIB.uw_mesh_table(self.handle, which, out.ctypes.data))
        return out

    def to_internal(self, W):
        """Original cell order -> internal order (numpy, [V, n])."""
        return np.ascontiguousarray(np.asarray(W)[:, self.old_of_new])

    def to_original(self, W):
        return np.asarray(W)[:, self.new_of_old]

    def _check_state(self, physics, **bufs):
        # host-only meshes (device < 0) are left to the library, which
        # rejects device calls on them
        nv = _nvar(physics)
        if self.device < 0 or nv is None:
            return
        for name, x in bufs.items():
            if name in ("t_dev", "dt_dev"):
                _device_buffer(x, self.device, 1, name, at_least=True)
            else:
                _device_buffer(x, self.device, nv * self.n_cells, name)

    def residual(self, physics: PhysicsC, W, L, stream=None, t=None):
        """L = L(W); at time t (moving-front boundaries) when t is given."""
        self._check_state(physics, W=W, L=L)
        if t is None:
            _check(LIB.uw_residual(self.handle, ctypes.byref(physics), _ptr(W), _ptr(L),
                                   _stream(stream)))
        else:
            _check(LIB.uw_residual_at(self.handle, ctypes.byref(physics), _ptr(W), _ptr(L),
                                      float(t), _stream(stream)))

    def residual_noalloc(self, physics: PhysicsC, W, L, stream=None):
        """L = L(W) without any device allocation (face states in the
        library's fixed per-device scratch; meshes up to 524288 cells in
        FP32 Euler); needs one earlier residual in the same precision."""
        self._check_state(physics, W=W, L=L)
        _check(LIB.uw_residual_noalloc(self.handle, ctypes.byref(physics), _ptr(W), _ptr(L),
                                       _stream(stream)))

    def rk3_step(self, physics: PhysicsC, W, t_dev, cfl=0.5, dt_fixed=0.0, t_end=float("inf"),
                 stream=None):
        self._check_state(physics, W=W, t_dev=t_dev)
        _check(LIB.uw_rk3_step(self.handle, ctypes.byref(physics), _ptr(W), cfl, dt_fixed, t_end,
                               _ptr(t_dev), _stream(stream)))

    def rk3_steps(self, physics: PhysicsC, W, t_dev, n_steps, cfl=0.5, dt_fixed=0.0,
                  t_end=float("inf"), stream=None):
        """n_steps SSP-RK3 steps in one call (one captured graph)."""
        self._check_state(physics, W=W, t_dev=t_dev)
        _check(LIB.uw_rk3_steps(self.handle, ctypes.byref(physics), _ptr(W), cfl, dt_fixed,
                                t_end, int(n_steps), _ptr(t_dev), _stream(stream)))

    def cfl_dt(self, physics: PhysicsC, W, cfl, dt_dev, stream=None):
        self._check_state(physics, W=W, dt_dev=dt_dev)
        _check(LIB.uw_cfl_dt(self.handle, ctypes.byref(physics), _ptr(W), cfl, _ptr(dt_dev),
                             _stream(stream)))

    def autotune(self, physics: PhysicsC, cache_path=None, stream=None):
        _check(LIB.uw_autotune(self.handle, None, ctypes.byref(physics),
                               None if cache_path is None else cache_path.encode(),
                               _stream(stream)))

    def check(self, stream=None):
        _check(LIB.uw_check(self.handle, None, _stream(stream)))

    def schedule(self, set_to=None):
        """The launch schedule (recon quads, recon triangles, flux): persistent
        blocks, 0 = one block per tile; a triangle entry of -1 reconstructs
        both cell types in one launch.  ``set_to`` (3 ints) replaces it
        first."""
        got = np.zeros(3, dtype=np.int32)
        s = None if set_to is None else np.ascontiguousarray(set_to, dtype=np.int32)
        _check(LIB.uw_schedule(self.handle, None, got.ctypes.data,
                               None if s is None else s.ctypes.data))
        return tuple(int(x) for x in got)

    def tile_size(self, set_to=0):
        """Cells per tile (256 or 512); ``set_to`` changes it first."""
        got = ctypes.c_int32(0)
        _check(LIB.uw_tile_size(self.handle, None, int(set_to), ctypes.byref(got)))
        return got.value

    def profile(self, enable=-1):
        """Returns ((recon_ms, flux_ms), (recon_count, flux_count)) recorded
        so far and clears them; enable = 1/0 switches recording on/off."""
        ms = np.zeros(2)
        cnt = np.zeros(2, dtype=np.int64)
        _check(LIB.uw_profile(self.handle, int(enable), ms.ctypes.data, cnt.ctypes.data))
        return tuple(ms), tuple(int(c) for c in cnt)


class Batch:
    """Several meshes advanced together; states concatenated per mesh."""

    def __init__(self, meshes, physics: PhysicsC):
        self.meshes = list(meshes)
        self.nvar = _nvar(physics)
        arr = (ctypes.c_void_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        h = ctypes.c_void_p()
        _check(LIB.uw_batch_create(arr, len(self.meshes), ctypes.byref(physics), ctypes.byref(h)))
        self.handle = h
        self.offsets = np.empty(len(self.meshes) + 1, dtype=np.int64)
        _check(LIB.uw_batch_offsets(h, self.offsets.ctypes.data))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and LIB is not None:
            LIB.uw_batch_destroy(h)
            self.handle = None

    def to_internal(self, states):
        """Per-instance states (original order, [V, n_k]) -> batch state [V, N]."""
        return np.ascontiguousarray(np.concatenate(
            [m.to_internal(W) for m, W in zip(self.meshes, states)], axis=1))

    def to_original(self, W):
        """Batch state [V, N] -> list of per-instance states in original order."""
        W = np.asarray(W)
        return [m.to_original(W[:, self.offsets[k]:self.offsets[k + 1]])
                for k, m in enumerate(self.meshes)]

    def rk3_step(self, W, t_dev, cfl=0.5, dt_fixed=0.0, t_end=float("inf"), n_steps=1,
                 stream=None):
        dev = self.meshes[0].device
        if dev >= 0 and self.nvar is not None:
            _device_buffer(W, dev, self.nvar * int(self.offsets[-1]), "W")
            _device_buffer(t_dev, dev, len(self.meshes), "t_dev", at_least=True)
        _check(LIB.uw_batch_rk3_step(self.handle, _ptr(W), cfl, dt_fixed, t_end, n_steps,
                                     _ptr(t_dev), _stream(stream)))

    def schedule(self, set_to=None):
        """As Mesh.schedule, for the batch's launches."""
        got = np.zeros(3, dtype=np.int32)
        s = None if set_to is None else np.ascontiguousarray(set_to, dtype=np.int32)
        _check(LIB.uw_schedule(None, self.handle, got.ctypes.data,
                               None if s is None else s.ctypes.data))
        return tuple(int(x) for x in got)

    def tile_size(self, set_to=0):
        """As Mesh.tile_size, for the batch."""
        got = ctypes.c_int32(0)
        _check(LIB.uw_tile_size(None, self.handle, int(set_to), ctypes.byref(got)))
        return got.value

    def autotune(self, physics: PhysicsC, cache_path=None, stream=None):
        _check(LIB.uw_autotune(None, self.handle, ctypes.byref(physics),
                               None if cache_path is None else cache_path.encode(),
                               _stream(stream)))

    def check(self, stream=None):
        _check(LIB.uw_check(None, self.handle, _stream(stream)))
