"""GPU parity of the checkpointed discrete adjoint (lbm_forward_checkpointed +
lbm_adjoint, and the torch.autograd wrapper) against the FP64 oracle adjoint,
which forms explicit 19x19 collision Jacobians and keeps every state.

Gradients of L(u(T)) with respect to the per-point force field and tau:
grad_F relative L2 error <= 1e-4, cosine >= 0.99999 and max elementwise
error <= 1e-3 of max |grad_F| on small lattices (FP32 arithmetic against
FP64), grad_tau relative error <= 1e-3.
Checkpoint spacing does not change the result at all (bitwise), because the
recomputed segments repeat the forward arithmetic exactly and the tau
reduction has a fixed order.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import near_rest_state, oracle_lattice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1309_1983_amd
    paper_1309_1983_amd.lib()


CASES = {
    # name: (shape, flags builder, lid velocity, force amplitude, tau)
    "duct_x4": ((12, 10, 9), lambda s: W.duct_flags(*s), (0, 0, 0), 1e-3, 0.7),
    "cavity_lid": ((13, 11, 10), lambda s: W.cavity_flags(*s), (0.05, 0.0, 0.02), 1e-3, 0.8),
    "random_moving": ((16, 8, 6), lambda s: W.random_flags(int(np.prod(s)), 7, 0.2, 0.05),
                      (0.03, -0.01, 0.02), 5e-4, 0.65),
    "periodic": ((8, 6, 5), lambda s: np.zeros(int(np.prod(s)), np.uint8), (0, 0, 0), 1e-3, 1.1),
    # 65 four-point groups per row: the forward recompute on the one-dimensional grid
    "wide_rows": ((260, 4, 3), lambda s: W.duct_flags(*s), (0, 0, 0), 1e-3, 0.7),
}


def _setup(name):
    shape, mk, uw, famp, tau = CASES[name]
    flags = mk(shape)
    N = flags.size
    F = W.random_force_field(N, 3, famp).astype(np.float32)
    s0 = near_rest_state(N, 4)
    g = W.random_velocity(N, 5, 1.0).astype(np.float32)
    g[:, flags != 0] = 0
    return shape, flags, uw, F, tau, s0, g


def _gpu_adjoint(shape, flags, uw, F, tau, s0, g, T, K, cells_per_lane=0):
    from paper_1309_1983_amd import Lattice
    lat = Lattice(*shape, tau, flags=flags, cells_per_lane=cells_per_lane)
    lat.set_wall_velocity(*uw)
    lat.set_force(torch.from_numpy(F))
    lat.set_populations(torch.from_numpy(s0))
    lat.forward_checkpointed(T, K)
    gF, gt = lat.adjoint(torch.from_numpy(g))
    out = gF.cpu().numpy().astype(np.float64)
    lat.close()
    return out, gt


def _compare(gF, gt, rF, rt, flags, tolF=1e-4, tolT=1e-3, tolE=1e-3):
    """grad_F: relative L2 error <= tolF and cosine >= 0.99999 (the adjoint
    tolerance fixed for FP32 against FP64), and element by element
    max |dgrad_F| / max |grad_F| <= tolE, so that a wrong value confined to a
    few points (e.g. wall links) cannot hide in the norm."""
    fl = flags == 0
    a, b = gF[:, fl].ravel(), rF[:, fl].ravel()
    rel = np.linalg.norm(a - b) / np.linalg.norm(b)
    cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
    elem = np.max(np.abs(a - b)) / np.max(np.abs(b))
    print(f"grad_F rel L2 {rel:.2e}, elementwise {elem:.2e}, cos {cos:.8f}; grad_tau {gt:.6e} vs {rt:.6e}")
    assert rel <= tolF and cos >= 0.99999
    assert elem <= tolE
    assert gt == pytest.approx(rt, rel=tolT)
    assert np.all(gF[:, ~fl] == 0)


@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_matches_oracle(name):
    shape, flags, uw, F, tau, s0, g = _setup(name)
    T, K = 12, 5          # segments of 5, 5 and 2 steps
    gF, gt = _gpu_adjoint(shape, flags, uw, F, tau, s0, g, T, K)
    olat = oracle_lattice(shape, tau, flags=flags, uw=uw, force_field=F)
    rF, rt = olat.adjoint(s0.astype(np.float64), T, g.astype(np.float64))
    _compare(gF, gt, rF, rt, flags)


def test_checkpoint_spacing_does_not_change_gradients():
    shape, flags, uw, F, tau, s0, g = _setup("duct_x4")
    T = 15
    ref = _gpu_adjoint(shape, flags, uw, F, tau, s0, g, T, T)
    for K in (1, 4, 7):
        got = _gpu_adjoint(shape, flags, uw, F, tau, s0, g, T, K)
        np.testing.assert_array_equal(got[0], ref[0])
        assert got[1] == ref[1]


@pytest.mark.parametrize("name", ["duct_x4", "random_moving", "periodic", "wide_rows"])
def test_vector_reverse_step_equals_one_point_reverse_step(name):
    """The two-points-per-work-item reverse step (and the four-point forward
    recompute) run the same per-point arithmetic as the one-point kernels:
    dL/dF agrees bit for bit; dL/dtau is summed per work-group in a different
    order, so it agrees to round-off."""
    shape, flags, uw, F, tau, s0, g = _setup(name)
    assert shape[0] % 4 == 0
    one = _gpu_adjoint(shape, flags, uw, F, tau, s0, g, 9, 4, cells_per_lane=1)
    vec = _gpu_adjoint(shape, flags, uw, F, tau, s0, g, 9, 4, cells_per_lane=0)
    np.testing.assert_array_equal(vec[0], one[0])
    assert vec[1] == pytest.approx(one[1], rel=1e-9)


def test_zero_steps_is_direct_term():
    shape, flags, uw, F, tau, s0, g = _setup("cavity_lid")
    gF, gt = _gpu_adjoint(shape, flags, uw, F, tau, s0, g, 0, 3)
    olat = oracle_lattice(shape, tau, flags=flags, uw=uw, force_field=F)
    rF, rt = olat.adjoint(s0.astype(np.float64), 0, g.astype(np.float64))
    fl = flags == 0
    np.testing.assert_allclose(gF[:, fl], rF[:, fl], rtol=1e-6, atol=0)
    assert gt == 0.0


def test_trajectory_invalidation():
    from paper_1309_1983_amd import LBMError, Lattice
    shape, flags, uw, F, tau, s0, g = _setup("duct_x4")
    lat = Lattice(*shape, tau, flags=flags)
    with pytest.raises(LBMError, match="STATE"):
        lat.adjoint(torch.from_numpy(g))
    lat.forward_checkpointed(4, 2)
    lat.adjoint(torch.from_numpy(g))
    lat.set_tau(0.75)
    with pytest.raises(LBMError, match="STATE"):
        lat.adjoint(torch.from_numpy(g))
    lat.forward_checkpointed(4, 2)
    lat.step(1)
    with pytest.raises(LBMError, match="STATE"):
        lat.adjoint(torch.from_numpy(g))
    lat.close()
    lat16 = Lattice(*shape, tau, flags=flags, storage="f16")
    with pytest.raises(LBMError, match="STATE"):
        lat16.forward_checkpointed(4, 2)
    lat16.close()


def test_autograd_rollout_matches_direct_adjoint():
    from paper_1309_1983_amd import Lattice, rollout
    shape, flags, uw, F, tau, s0, _ = _setup("duct_x4")
    N = flags.size
    fl = torch.from_numpy(flags == 0).cuda()
    target = torch.from_numpy(W.random_velocity(N, 9, 1e-3).astype(np.float32)).cuda()
    lat = Lattice(*shape, tau, flags=flags)
    lat.set_populations(torch.from_numpy(s0))
    force = torch.from_numpy(F).cuda().requires_grad_(True)
    tau_t = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    s0_t = torch.from_numpy(s0).cuda()
    u = rollout(lat, force, tau_t, T=10, K=3, s0=s0_t)
    loss = ((u - target)[:, fl] ** 2).sum() / fl.sum()
    loss.backward()
    g = torch.zeros(3, N, device="cuda")
    g[:, fl] = (2 * (u - target)[:, fl] / fl.sum()).detach()
    olat = oracle_lattice(shape, tau, flags=flags, force_field=F)
    rF, rt = olat.adjoint(s0.astype(np.float64), 10, g.cpu().numpy().astype(np.float64))
    _compare(force.grad.cpu().numpy().astype(np.float64), float(tau_t.grad), rF, rt, flags)
    lat.close()


def test_adjoint_config_64cube_vs_oracle_and_fd():
    """The 64^3 periodic-z duct with a per-point force (|F| <= 1e-5), tau 0.7,
    T = 200, checkpoint every 20: loss = mean squared velocity error against
    the u(T) of a second force field. GPU gradients vs the FP64 oracle
    adjoint, and a coarse central difference in tau on the GPU."""
    from paper_1309_1983_amd import Lattice
    n, tau, T, K = 64, 0.7, 200, 20
    flags = W.duct_flags(n, n, n)
    N = flags.size
    fl = flags == 0
    F = W.random_force_field(N, 1, 1e-5).astype(np.float32)
    F2 = W.random_force_field(N, 2, 1e-5).astype(np.float32)
    s0 = oracle.init_equilibrium(N).astype(np.float32)   # rest
    # target from the oracle with the second force field
    ot = oracle_lattice((n, n, n), tau, flags=flags, force_field=F2)
    ustar = ot.macros(ot.run(s0.astype(np.float64), T))[1].astype(np.float32)

    lat = Lattice(n, n, n, tau, flags=flags)
    lat.set_force(torch.from_numpy(F))
    lat.set_populations(torch.from_numpy(s0))
    lat.forward_checkpointed(T, K)
    _, u = lat.macros()
    u = u.cpu().numpy().astype(np.float64)
    g = np.zeros((3, N))
    g[:, fl] = 2 * (u - ustar)[:, fl] / fl.sum()
    gF, gt = lat.adjoint(torch.from_numpy(g.astype(np.float32)))
    gF = gF.cpu().numpy().astype(np.float64)
    loss_gpu = ((u - ustar)[:, fl] ** 2).sum() / fl.sum()

    of = oracle_lattice((n, n, n), tau, flags=flags, force_field=F)
    uo = of.macros(of.run(s0.astype(np.float64), T))[1]
    go = np.zeros((3, N))
    go[:, fl] = 2 * (uo - ustar)[:, fl] / fl.sum()
    rF, rt = of.adjoint(s0.astype(np.float64), T, go)
    loss_ref = ((uo - ustar)[:, fl] ** 2).sum() / fl.sum()
    print(f"loss gpu {loss_gpu:.6e} oracle {loss_ref:.6e}")
    assert loss_gpu == pytest.approx(loss_ref, rel=1e-3)
    _compare(gF, gt, rF, rt, flags, tolF=1e-3, tolT=1e-3)

    # coarse GPU central difference in tau
    def loss_at(t):
        lat.set_tau(t)
        lat.set_populations(torch.from_numpy(s0))
        lat.step(T)
        uu = lat.macros()[1].cpu().numpy().astype(np.float64)
        return ((uu - ustar)[:, fl] ** 2).sum() / fl.sum()
    h = 1e-2 * tau
    fd = (loss_at(tau + h) - loss_at(tau - h)) / (2 * h)
    lat.close()
    print(f"grad_tau adjoint {gt:.6e}, GPU central difference {fd:.6e}")
    assert gt == pytest.approx(fd, rel=0.05)


@pytest.mark.timeout(600)
def test_adjoint_256cube_checkpoint_invariance_and_fd():
    """The adjoint at the benchmarked size: 256^3 duct with a per-point force,
    tau 0.7, T = 200. Checkpoints every 50 and every 40 steps give bitwise
    equal gradients, and dL/dtau agrees with a GPU central difference."""
    from paper_1309_1983_amd import Lattice
    n, tau, T = 256, 0.7, 200
    flags = W.duct_flags(n, n, n)
    N = flags.size
    fl = torch.from_numpy(flags == 0).cuda()
    F = torch.from_numpy(W.random_force_field(N, 1, 1e-5).astype(np.float32)).cuda()
    target = torch.from_numpy(W.random_velocity(N, 2, 1e-5).astype(np.float32)).cuda()
    lat = Lattice(n, n, n, tau, flags=flags)
    lat.set_force(F)
    s0 = lat.populations()

    def loss_and_grad(K):
        lat.set_populations(s0)
        lat.forward_checkpointed(T, K)
        _, u = lat.macros()
        d = (u - target)[:, fl]
        loss = float((d.double() ** 2).sum() / fl.sum())
        g = torch.zeros(3, N, device="cuda")
        g[:, fl] = 2 * d / fl.sum()
        gF, gt = lat.adjoint(g)
        return loss, gF, gt

    loss, gF50, gt50 = loss_and_grad(50)
    _, gF40, gt40 = loss_and_grad(40)
    assert torch.equal(gF50, gF40) and gt50 == gt40

    def loss_at(t):
        lat.set_tau(t)
        lat.set_populations(s0)
        lat.step(T)
        _, u = lat.macros()
        return float((((u - target)[:, fl]).double() ** 2).sum() / fl.sum())
    h = 1e-2 * tau
    fd = (loss_at(tau + h) - loss_at(tau - h)) / (2 * h)
    lat.close()
    print(f"256^3: loss {loss:.6e}, dL/dtau adjoint {gt50:.6e}, GPU central difference {fd:.6e}")
    assert gt50 == pytest.approx(fd, rel=0.05)


def test_one_point_reverse_step_on_512_point_rows():
    """Rows that are a multiple of 512 points take 512-point work-groups for
    the forward one-point kernels; the one-point reverse step caps its groups
    at its 256-work-item bound and matches the two-point reverse step."""
    shape, tau = (512, 2, 2), 0.8
    N = int(np.prod(shape))
    flags = W.random_flags(N, 17, 0.2, 0.05)
    F = W.random_force_field(N, 18, 1e-3).astype(np.float32)
    s0 = near_rest_state(N, 19)
    g = W.random_velocity(N, 20, 1.0).astype(np.float32)
    g[:, flags != 0] = 0
    uw = (0.03, 0.0, -0.01)
    one = _gpu_adjoint(shape, flags, uw, F, tau, s0, g, 6, 4, cells_per_lane=1)
    vec = _gpu_adjoint(shape, flags, uw, F, tau, s0, g, 6, 4, cells_per_lane=0)
    np.testing.assert_array_equal(vec[0], one[0])
    assert vec[1] == pytest.approx(one[1], rel=1e-9)
    olat = oracle_lattice(shape, tau, flags=flags, uw=uw, force_field=F)
    rF, rt = olat.adjoint(s0.astype(np.float64), 6, g.astype(np.float64))
    _compare(one[0], one[1], rF, rt, flags)


def test_autograd_force_shapes():
    """rollout() takes the force field in any shape holding 3*N values and
    returns its gradient in that shape; a 3-vector is rejected."""
    from paper_1309_1983_amd import Lattice, rollout
    shape, flags, uw, F, tau, s0, _ = _setup("duct_x4")
    N = flags.size
    nx, ny, nz = shape
    lat = Lattice(*shape, tau, flags=flags)
    s0_t = torch.from_numpy(s0).cuda()
    grads = []
    for fshape in ((3, N), (3, nz, ny, nx)):
        force = torch.from_numpy(F).cuda().reshape(fshape).clone().requires_grad_(True)
        tau_t = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
        u = rollout(lat, force, tau_t, T=6, K=3, s0=s0_t)
        (u[:, torch.from_numpy(flags == 0).cuda()] ** 2).sum().backward()
        assert force.grad.shape == force.shape
        grads.append(force.grad.reshape(3, N))
    assert torch.equal(grads[0], grads[1])
    with pytest.raises(ValueError, match="3\\*N"):
        rollout(lat, torch.zeros(3, device="cuda", requires_grad=True),
                torch.tensor(tau, dtype=torch.float64), T=2, K=1, s0=s0_t)
    lat.close()
