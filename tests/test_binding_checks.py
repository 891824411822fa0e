"""The binding's checks of device arguments (host logic, no GPU): the C-ABI
cannot check device pointers, so a wrong tensor must be refused before its
address reaches the library."""
import numpy as np
import pytest
import torch


@pytest.fixture(scope="module")
def uw():
    import paper_1712_08317_amd as mod
    return mod


def test_wrong_arguments_are_refused_in_order(uw):
    chk = uw._device_buffer
    with pytest.raises(ValueError, match="torch tensor"):
        chk(np.zeros(8), 0, 8, "W")
    with pytest.raises(ValueError, match="float64"):
        chk(torch.zeros(8, dtype=torch.float32), 0, 8, "W")
    with pytest.raises(ValueError, match="contiguous"):
        chk(torch.zeros(4, 4, dtype=torch.float64).t(), 0, 16, "W")
    with pytest.raises(ValueError, match="hold 9 values, has 8"):
        chk(torch.zeros(8, dtype=torch.float64), 0, 9, "W")
    with pytest.raises(ValueError, match="at least 3"):
        chk(torch.zeros(2, dtype=torch.float64), 0, 3, "t_dev", at_least=True)
    # right type, size and layout, but in host memory
    with pytest.raises(ValueError, match="must be on cuda:0"):
        chk(torch.zeros(8, dtype=torch.float64), 0, 8, "W")
    with pytest.raises(ValueError, match="must be on cuda:1"):
        chk(torch.zeros(4, dtype=torch.float64), 1, 2, "t_dev", at_least=True)


def test_variables_per_equation(uw):
    assert uw._nvar(uw.make_physics(uw.UW_EULER)) == 4
    assert uw._nvar(uw.make_physics(uw.UW_ADVECTION)) == 1
    assert uw._nvar(uw.make_physics(7)) is None


def test_host_only_meshes_leave_the_check_to_the_library(uw):
    """A mesh without a device: the library itself refuses the call."""
    import workloads as wl
    M = uw.Mesh.from_workload(wl.mesh_c1(n=6), device=-1)
    M.precompute()
    W = torch.zeros(M.n_cells, dtype=torch.float32)      # wrong in every way
    with pytest.raises(uw.UwError) as e:
        M.residual(uw.make_physics(uw.UW_ADVECTION), W, W.clone(), stream=0)
    assert e.value.status == uw.UW_ESTATE
