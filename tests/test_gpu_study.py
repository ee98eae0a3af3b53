"""GPU checks of the memory-access study kernels (include/lbm_study.h).

- streams and offset-by-one propagations move exactly the expected elements;
- the one-point pull iteration (Algorithm 3) equals the library's step bit
  for bit, and the push iteration (Algorithm 2) evolves the same recurrence:
  push(P s) = P pull(s) bit for bit, P being streaming with bounce-back;
- both match the FP64 oracle after 50 steps (max |df|/|f| <= 1e-5).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import fluid_rel_err, near_rest_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1309_1983_amd
    paper_1309_1983_amd.lib()


@pytest.mark.parametrize("width", [1, 4])
@pytest.mark.parametrize("nvec", [1, 4, 19])
@pytest.mark.parametrize("roff,woff", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_stream_modes_move_the_right_elements(width, nvec, roff, woff):
    from paper_1309_1983_amd import study
    n = 4096 + 8
    g = torch.Generator(device="cuda").manual_seed(nvec * 10 + roff * 2 + woff)
    src = torch.rand(nvec, n, device="cuda", generator=g)
    dst = torch.zeros(nvec, n, device="cuda")
    study.stream("copy", src, dst, None, n, nvec, roff, woff, width)
    assert torch.equal(dst[:, woff:woff + n - 1], src[:, roff:roff + n - 1])
    sink = torch.zeros(n, device="cuda")
    study.stream("read", src, None, sink, n, nvec, roff, 0, width)
    ref = src[:, roff:roff + n - 1].double().sum(0)
    assert torch.allclose(sink[:n - 1].double(), ref, rtol=1e-5, atol=1e-5)
    dst.zero_()
    study.stream("write", None, dst, None, n, nvec, 0, woff, width)
    k = torch.arange(n - 1, device="cuda", dtype=torch.float32)
    v = torch.arange(nvec, device="cuda", dtype=torch.float32)[:, None]
    assert torch.equal(dst[:, woff:woff + n - 1], k[None, :] + v)


@pytest.mark.parametrize("shape", [(256, 6, 5), (36, 7, 3), (1028, 2, 2)])
def test_plane_streams_move_the_right_elements(shape):
    """The 19-plane stream kernel: copy is exact, write stores the stated
    pattern, read leaves the sink alone (its guard never fires)."""
    from paper_1309_1983_amd import study
    nx, ny, nz = shape
    N = nx * ny * nz
    g = torch.Generator(device="cuda").manual_seed(nx)
    src = torch.rand(19 * N, device="cuda", generator=g)
    dst = torch.zeros(19 * N, device="cuda")
    study.planes("copy", src, dst, None, nx, ny, nz)
    assert torch.equal(dst, src)
    sink = torch.full((4,), 7.0, device="cuda")
    study.planes("read", src, None, sink, nx, ny, nz)
    assert torch.equal(sink, torch.full((4,), 7.0, device="cuda"))
    dst.zero_()
    study.planes("write", None, dst, None, nx, ny, nz)
    v = dst.view(nz, 19, ny * nx // 4, 4)
    i = torch.arange(19, device="cuda", dtype=torch.float32).view(1, 19, 1)
    o = (4 * torch.arange(ny * nx // 4, device="cuda", dtype=torch.float32)).view(1, 1, -1)
    assert torch.equal(v[..., 0], i.expand(nz, 19, ny * nx // 4))
    assert torch.equal(v[..., 1], o.expand(nz, 19, ny * nx // 4))
    assert torch.all(v[..., 2] == 0) and torch.all(v[..., 3] == 1)


@pytest.mark.parametrize("method", ["direct", "lds", "dpp", "direct4"])
@pytest.mark.parametrize("nx", [64, 256, 1024])
def test_shift_methods_are_a_periodic_roll(method, nx):
    from paper_1309_1983_amd import study
    rows = 37
    src = torch.rand(rows, nx, device="cuda", generator=torch.Generator(device="cuda").manual_seed(nx))
    dst = torch.full_like(src, -1.0)
    study.shift(src, dst, nx, rows, method)
    assert torch.equal(dst, torch.roll(src, 1, dims=1))


def _study_run(scheme, shape, flags, tau, f0, steps, block_x=64):
    from paper_1309_1983_amd import study
    nx, ny, nz = shape
    a = torch.from_numpy(f0).cuda()
    b = torch.zeros_like(a)
    fl = torch.from_numpy(flags).cuda()
    for _ in range(steps):
        study.step(a, b, fl, nx, ny, nz, tau, scheme, block_x)
        a, b = b, a
    torch.cuda.synchronize()
    return a.cpu().numpy()


def _library_stream(shape, flags, f):
    from paper_1309_1983_amd import Lattice
    lat = Lattice(*shape, 0.8, flags=flags, cells_per_lane=1)
    lat.set_populations(torch.from_numpy(f))
    lat.stream_only(1)
    out = lat.populations().cpu().numpy()
    lat.close()
    return out


@pytest.mark.parametrize("shape,solid", [((33, 17, 11), 0.15), ((64, 16, 8), 0.0)])
def test_push_and_pull_evolve_the_same_recurrence(shape, solid):
    from paper_1309_1983_amd import Lattice
    N = int(np.prod(shape))
    flags = W.random_flags(N, seed=5, solid_fraction=solid)
    tau = 0.75
    s0 = near_rest_state(N, 6)
    fl = flags == 0
    steps = 7
    pull = _study_run("pull", shape, flags, tau, s0, steps)
    lat = Lattice(*shape, tau, flags=flags, cells_per_lane=1)
    lat.set_populations(torch.from_numpy(s0))
    lat.step(steps)
    lib = lat.populations().cpu().numpy()
    lat.close()
    np.testing.assert_array_equal(pull[:, fl], lib[:, fl])
    p0 = _library_stream(shape, flags, s0)
    push = _study_run("push", shape, flags, tau, p0, steps)
    np.testing.assert_array_equal(push[:, fl], _library_stream(shape, flags, pull)[:, fl])


def test_push_and_pull_match_oracle():
    shape, tau, steps = (40, 24, 20), 0.7, 50
    N = int(np.prod(shape))
    flags = W.cavity_flags(*shape)
    flags[flags == 2] = 1   # the study kernels have resting walls only
    s0 = near_rest_state(N, 8)
    olat = oracle.Lattice(*shape, float(np.float32(tau)), flags=flags)
    ref = olat.run(s0.astype(np.float64), steps)
    pull = _study_run("pull", shape, flags, tau, s0, steps)
    assert fluid_rel_err(pull.astype(np.float64), ref, flags) <= 1e-5
    p0 = olat.step(s0.astype(np.float64), collide=False).astype(np.float32)
    push = _study_run("push", shape, flags, tau, p0, steps)
    p_ref = olat.step(ref, collide=False)
    assert fluid_rel_err(push.astype(np.float64), p_ref, flags) <= 1e-5
