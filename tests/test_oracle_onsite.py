"""Pins of the oracle's on-site velocity nodes (the boundary family of the
paper's cavity validation, Section 5; flags 3 and 4).

The node lies on the wall and carries a prescribed velocity; the populations
arriving from solid cells are rebuilt so that the node holds mass rho and
bare momentum rho*u - F/2. These tests tie that reading to facts fixed
outside the oracle's own formulas:

- plane Couette flow between on-site walls is exactly linear and plane
  Poiseuille flow exactly parabolic, with zero velocity on the node planes
  (the closed-form steady solutions of the Navier-Stokes equations that this
  boundary family reproduces to round-off);
- a uniform flow matching the prescribed velocity on every face, edge and
  corner of a closed box is a fixed point, and so is the rest state;
- every on-site node carries its prescribed velocity after every step, with
  body force and arbitrary interior flow;
- a lid moving along x gives a flow that is mirror-symmetric in z;
- the square-duct flow converges to the Fourier-series solution at second
  order (this exercises the edge nodes of the duct's corners);
- stream-only steps ignore the on-site reconstruction (nodes are plain fluid).
"""
import numpy as np
import pytest

import oracle
import workloads as W

Q = 19


def _solid(flags):
    return (flags == W.WALL) | (flags == W.MOVING_WALL)


def _steady_channel(h, tau, uw=(0, 0, 0), force=None, lid=False, tdiff=25):
    flags = W.onsite_channel_flags(h, lid=lid)
    ny = h + 3
    lat = oracle.Lattice(1, ny, 1, tau, flags=flags, uw=uw, force=force)
    nu = (tau - 0.5) / 3
    steps = int(tdiff * h * h / nu)
    s = lat.run(oracle.init_equilibrium(ny), steps)
    rho, u = lat.macros(s)
    return flags, rho, u, np.arange(ny) - 1.0   # distance from the lower node plane


def test_onsite_couette_is_exactly_linear():
    h, U = 8, 0.05
    flags, rho, u, sy = _steady_channel(h, 0.8, uw=(U, 0, 0), lid=True)
    fl = ~_solid(flags)
    exact = U * sy / h
    err = np.max(np.abs(u[0, fl] - exact[fl])) / U
    assert err <= 1e-12
    assert np.max(np.abs(u[1:, fl])) <= 1e-15


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0, 1.5])
def test_onsite_poiseuille_is_exactly_parabolic(tau):
    """u(s) = F s (h - s) / (2 nu), s the distance from the lower node plane:
    no slip on the node planes, unlike halfway bounce-back."""
    h, F = 8, 1e-5
    nu = (tau - 0.5) / 3
    flags, rho, u, sy = _steady_channel(h, tau, force=(F, 0, 0))
    fl = ~_solid(flags)
    exact = F * sy * (h - sy) / (2 * nu)
    err = np.max(np.abs(u[0, fl] - exact[fl])) / exact.max()
    assert err <= 1e-9
    assert np.max(np.abs(u[0, flags == W.ONSITE])) <= 1e-15


def test_onsite_uniform_flow_is_a_fixed_point():
    """Every face, edge and corner node prescribes the same velocity U, which
    has components along all three axes; f = f^eq(1, U) must not change."""
    shape = (9, 8, 7)
    N = int(np.prod(shape))
    flags = W.onsite_cavity_flags(*shape)
    flags[flags == W.ONSITE] = W.ONSITE_MOVING
    U = np.array([0.04, -0.03, 0.02])
    lat = oracle.Lattice(*shape, 0.7, flags=flags, uw=U)
    s0 = oracle.init_equilibrium(N, np.ones(N), np.repeat(U[:, None], N, axis=1))
    s = lat.run(s0, 40)
    fl = ~_solid(flags)
    assert np.max(np.abs(s - s0)[:, fl]) <= 1e-14


def test_onsite_rest_is_a_fixed_point():
    shape = (9, 8, 7)
    N = int(np.prod(shape))
    flags = W.onsite_cavity_flags(*shape)
    lat = oracle.Lattice(*shape, 0.6, flags=flags)
    s0 = oracle.init_equilibrium(N)
    s = lat.run(s0, 40)
    assert np.max(np.abs(s - s0)[:, ~_solid(flags)]) <= 1e-15


def test_onsite_nodes_carry_the_prescribed_velocity():
    """Random start, per-point body force, lid velocity with all three
    components: after the steps every on-site node reports exactly its
    prescribed velocity (macroscopic u includes the Guo half-force)."""
    shape = (9, 8, 7)
    N = int(np.prod(shape))
    flags = W.onsite_cavity_flags(*shape)
    F = W.random_force_field(N, 3, 1e-4)
    uw = np.array([0.05, 0.01, -0.02])
    lat = oracle.Lattice(*shape, 0.65, flags=flags, uw=uw, force_field=F)
    s0 = oracle.init_equilibrium(N, W.random_density(N, 4, 0.01), W.random_velocity(N, 5, 0.02))
    s = s0
    for _ in range(3):
        s = lat.run(s, 10)
        _, u = lat.macros(s)
        assert np.max(np.abs(u[:, flags == W.ONSITE])) <= 1e-14
        assert np.max(np.abs(u[:, flags == W.ONSITE_MOVING] - uw[:, None])) <= 1e-14


def test_onsite_cavity_is_mirror_symmetric_in_z():
    shape = (10, 9, 8)
    nx, ny, nz = shape
    flags = W.onsite_cavity_flags(*shape)
    lat = oracle.Lattice(*shape, 0.6, flags=flags, uw=(0.08, 0, 0))
    s = lat.run(oracle.init_equilibrium(nx * ny * nz), 200)
    _, u = lat.macros(s)
    u = u.reshape(3, nz, ny, nx)
    assert np.abs(u[2]).max() > 1e-4             # a genuinely 3-D flow
    assert np.max(np.abs(u[0] - u[0][::-1])) <= 1e-14
    assert np.max(np.abs(u[1] - u[1][::-1])) <= 1e-14
    assert np.max(np.abs(u[2] + u[2][::-1])) <= 1e-14


def _duct_series(h, F, nu, X, Y, terms=100):
    """Fully developed flow in a square duct of side h (walls on the node
    planes 0 and h) driven by body force F along the axis: the classical
    Fourier series of the Poisson problem nu * lap(u) = -F, u = 0 on the
    walls."""
    a = h / 2.0
    x, y = X - a, np.abs(Y - a)
    u = np.zeros_like(x)
    for k in range(terms):
        m = 2 * k + 1
        A, B = m * np.pi * y / (2 * a), m * np.pi / 2
        ratio = np.exp(A - B) * (1 + np.exp(-2 * A)) / (1 + np.exp(-2 * B))   # cosh A / cosh B
        u += (-1) ** k * (1 - ratio) * np.cos(m * np.pi * x / (2 * a)) / m ** 3
    return 16 * F * a * a / (nu * np.pi ** 3) * u


def test_onsite_square_duct_converges_at_second_order():
    tau, F = 0.8, 1e-5
    nu = (tau - 0.5) / 3
    errs = []
    for h in (4, 8, 16):
        n = h + 3
        f = np.zeros((1, n, n), np.uint8)
        f[0, 1:-1, 1:-1] = W.ONSITE
        f[0, 2:-2, 2:-2] = W.FLUID
        f[0, 0, :] = f[0, -1, :] = f[0, :, 0] = f[0, :, -1] = W.WALL
        flags = f.reshape(-1)
        lat = oracle.Lattice(n, n, 1, tau, flags=flags, force=(0, 0, F))
        s = lat.run(oracle.init_equilibrium(n * n), int(12 * h * h / nu))
        _, u = lat.macros(s)
        Y, X = np.meshgrid(np.arange(n) - 1.0, np.arange(n) - 1.0, indexing="ij")
        inside = ~_solid(flags).reshape(n, n)
        ex = _duct_series(h, F, nu, X, Y)
        errs.append(np.max(np.abs(u[2].reshape(n, n) - ex)[inside]) / ex[inside].max())
    assert errs[1] <= 0.02
    assert errs[0] / errs[1] >= 3.5 and errs[1] / errs[2] >= 3.5


def test_stream_only_treats_onsite_nodes_as_fluid():
    shape = (7, 8, 6)
    N = int(np.prod(shape))
    flags = W.onsite_cavity_flags(*shape)
    plain = flags.copy()
    plain[(plain == W.ONSITE) | (plain == W.ONSITE_MOVING)] = W.FLUID
    s0 = W.random_values(Q * N, 9).reshape(Q, N)
    a = oracle.Lattice(*shape, 0.7, flags=flags, uw=(0.1, 0, 0)).run(s0, 5, collide=False)
    b = oracle.Lattice(*shape, 0.7, flags=plain, uw=(0.1, 0, 0)).run(s0, 5, collide=False)
    np.testing.assert_array_equal(a, b)


def test_oracle_adjoint_rejects_onsite_nodes():
    shape = (6, 6, 5)
    N = int(np.prod(shape))
    lat = oracle.Lattice(*shape, 0.7, flags=W.onsite_cavity_flags(*shape))
    with pytest.raises(ValueError, match="on-site"):
        lat.adjoint(oracle.init_equilibrium(N), 2, np.zeros((3, N)))
