"""uw_residual_noalloc, the residual that allocates no device memory (its
face states live in a fixed per-device scratch array), against uw_residual
through the C-ABI: bit-identical results on two calls in a row, the second
on a smaller mesh (the scratch still holds the first call's values); the
precondition and the size limit are refused before any launch."""
import ctypes

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _call(fn, M, ph, W, L):
    import torch
    st = torch.cuda.current_stream().cuda_stream
    return fn(M.handle, ctypes.byref(ph), ctypes.c_void_p(W.data_ptr()),
              ctypes.c_void_p(L.data_ptr()), ctypes.c_void_p(st))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_residual_equals_residual(prec):
    import torch
    import paper_1712_08317_amd as uw
    ph = uw.make_physics(uw.UW_EULER, precision=uw.UW_FP64 if prec == "fp64" else uw.UW_FP32)
    meshes = [wl.mesh_c5(n=64, block=16, jitter=0.3, seed=7),          # 6144 mixed cells
              wl.grid_mesh(9, 9, 2.0, 2.0, "tri", 0.2, 8, True)]      # 162 triangles
    runs = []
    for k, mesh in enumerate(meshes):
        M = uw.Mesh.from_workload(mesh, device=0)
        M.precompute()
        W = torch.from_numpy(M.to_internal(wl.seeded_state(mesh, 4, 3 + k))).to("cuda:0")
        ref = torch.empty_like(W)
        got = torch.full_like(W, float("nan"))
        print(prec, "mesh", k, M.n_cells, "cells", flush=True)
        # the tables of this precision are not on the device before a first
        # allocating call: refused, nothing launched
        assert _call(uw.LIB.uw_residual_noalloc, M, ph, W, got) == uw.UW_ESTATE
        assert _call(uw.LIB.uw_residual, M, ph, W, ref) == uw.UW_OK
        runs.append((M, W, ref, got))
    torch.cuda.synchronize()
    for M, W, ref, got in runs:          # two calls in a row, larger mesh first
        assert _call(uw.LIB.uw_residual_noalloc, M, ph, W, got) == uw.UW_OK
    torch.cuda.synchronize()
    for M, W, ref, got in runs:
        M.check()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref)
    # and once more on the larger mesh, after the smaller one
    M, W, ref, got = runs[0]
    got.fill_(float("nan"))
    assert _call(uw.LIB.uw_residual_noalloc, M, ph, W, got) == uw.UW_OK
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


def test_noalloc_residual_size_limit():
    """270,400 cells: FP64 Euler face states need 69.2 MB > 64 MiB, refused
    before any launch (UW_EINVAL); FP32 needs 34.6 MB (runs, equal to
    uw_residual)."""
    import torch
    import paper_1712_08317_amd as uw
    mesh = wl.grid_mesh(520, 520, 2.0, 2.0, "quad", 0.2, 9, True)
    M = uw.Mesh.from_workload(mesh, device=0)
    M.precompute()
    W = torch.from_numpy(M.to_internal(wl.initial_state("c2q", mesh, q=2))).to("cuda:0")
    for prec, ok in ((uw.UW_FP64, False), (uw.UW_FP32, True)):
        ph = uw.make_physics(uw.UW_EULER, precision=prec)
        ref = torch.empty_like(W)
        got = torch.full_like(W, float("nan"))
        assert _call(uw.LIB.uw_residual, M, ph, W, ref) == uw.UW_OK
        st = _call(uw.LIB.uw_residual_noalloc, M, ph, W, got)
        torch.cuda.synchronize()
        if ok:
            assert st == uw.UW_OK
            assert torch.equal(got, ref)
        else:
            assert st == uw.UW_EINVAL
            assert "scratch" in uw.LIB.uw_last_error().decode()
            assert torch.isnan(got).all()
    M.check()
