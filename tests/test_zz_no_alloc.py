"""The allocation-free adjoint entry point (lbm_adjoint_noalloc), called
through the C ABI, gives the same gradients as lbm_adjoint: dL/dF bit for
bit and dL/dtau bit for bit (the per-work-group partials are summed in the
same order). Two calls in a row, the second on a smaller lattice, so that the
shared scratch array's leftovers from the first call must not leak into the
second; lattices above its 2^18-point limit are refused."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_common import near_rest_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1309_1983_amd
    paper_1309_1983_amd.lib()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(shape, seed, T, K, noalloc_first, **kw):
    from paper_1309_1983_amd import Lattice, _abi
    N = int(np.prod(shape))
    flags = W.random_flags(N, seed, 0.15, 0.05)
    F = torch.from_numpy(W.random_force_field(N, seed + 1, 1e-3).astype(np.float32))
    s0 = torch.from_numpy(near_rest_state(N, seed + 2))
    g = W.random_velocity(N, seed + 3, 1.0).astype(np.float32)
    g[:, flags != 0] = 0
    g = torch.from_numpy(g).cuda()
    lat = Lattice(*shape, 0.7, flags=flags, **kw)
    lat.set_wall_velocity(0.03, -0.01, 0.02)
    lat.set_force(F)
    lat.set_populations(s0)
    lat.forward_checkpointed(T, K)

    def noalloc():
        gF = torch.full((3, N), float("nan"), device="cuda")
        gt = ctypes.c_double(float("nan"))
        _abi.call("lbm_adjoint_noalloc", lat._h, _ptr(g), _ptr(gF), ctypes.byref(gt))
        return gF.cpu(), gt.value

    def library():
        gF, gt = lat.adjoint(g)
        return gF.cpu(), gt

    if noalloc_first:
        a = noalloc()
        b = library()
    else:
        b = library()
        a = noalloc()
    bytes_before = lat.device_bytes()
    again = noalloc()
    assert lat.device_bytes() == bytes_before      # the entry point allocated nothing
    lat.close()
    return a, b, again


def test_noalloc_adjoint_equals_adjoint_two_calls():
    # first call on a 64^3-sized lattice (the limit), the second smaller
    cases = [((64, 64, 64), 7, 12, 5, False, {}), ((20, 14, 11), 9, 9, 4, True, {}),
             ((17, 8, 6), 11, 6, 3, True, {"cells_per_lane": 1})]
    for shape, seed, T, K, first, kw in cases:
        a, b, again = _both(shape, seed, T, K, first, **kw)
        assert torch.equal(a[0], b[0]), shape
        assert a[1] == b[1], (shape, a[1], b[1])
        assert torch.equal(again[0], a[0]) and again[1] == a[1]
        assert torch.isfinite(a[0]).all()
        print(f"{shape}: dL/dtau {a[1]:.9e} from both entry points")


def test_noalloc_adjoint_rejects_large_lattices_and_missing_trajectory():
    from paper_1309_1983_amd import LBMError, Lattice, _abi
    lat = Lattice(65, 64, 64, 0.7)
    N = lat.N
    g = torch.zeros(3, N, device="cuda")
    gF = torch.empty(3, N, device="cuda")
    gt = ctypes.c_double()
    lat.forward_checkpointed(2, 1)
    with pytest.raises(LBMError, match="INVALID.*at most"):
        _abi.call("lbm_adjoint_noalloc", lat._h, _ptr(g), _ptr(gF), ctypes.byref(gt))
    lat.close()
    lat = Lattice(16, 8, 8, 0.7)
    g = torch.zeros(3, lat.N, device="cuda")
    gF = torch.empty(3, lat.N, device="cuda")
    with pytest.raises(LBMError, match="STATE"):
        _abi.call("lbm_adjoint_noalloc", lat._h, _ptr(g), _ptr(gF), ctypes.byref(gt))
    lat.close()
