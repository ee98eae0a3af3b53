"""Pins of the oracle's full step against what the method fixes.

- streaming is an exact permutation (np.roll brute force; return to the
  initial state after a full period, also through bounce-back walls);
- rest is a fixed point; mass and momentum are conserved, and a uniform Guo
  force adds exactly t * N_fluid * F of momentum;
- the shear viscosity is nu = (tau - 1/2)/3 (the scaling of Eq. (8)):
  shear-wave and Taylor-Green decay;
- plane Poiseuille flow with halfway bounce-back reaches the exact discrete
  parabola with its tau-dependent slip; Couette flow is exactly linear.
"""
import numpy as np
import pytest

import workloads as W


def _rest(orc, N):
    return orc.init_equilibrium(N)


def test_stream_only_is_np_roll(orc):
    """Periodic box, no walls: one pull step moves population i by +e_i."""
    E, _, _ = orc.tables()
    nx, ny, nz = 5, 4, 3
    N = nx * ny * nz
    s = W.random_values((19, N), seed=1, dtype=np.float64)
    L = orc.Lattice(nx, ny, nz, 0.8)
    out = L.step(s, collide=False)
    for i in range(19):
        grid = s[i].reshape(nz, ny, nx)
        ref = np.roll(grid, shift=(E[i, 2], E[i, 1], E[i, 0]), axis=(0, 1, 2)).reshape(-1)
        np.testing.assert_array_equal(out[i], ref)


def test_stream_only_full_period_is_identity(orc):
    L_ = 6
    s = W.random_values((19, L_ ** 3), seed=2, dtype=np.float64)
    L = orc.Lattice(L_, L_, L_, 0.8)
    np.testing.assert_array_equal(L.run(s, L_, collide=False), s)


def test_stream_only_through_walls_returns_after_2n(orc):
    """Channel with walls at y = 0 and y = n + 1: every population travels to
    a wall, is reversed by bounce-back and retraces its path, so 2n pure
    streaming steps are the identity on the fluid cells when nx and nz divide
    2n. A wrong opposite or source index breaks this."""
    n = 5
    nx = nz = 10
    flags = W.channel_flags(n, nx, nz)
    N = flags.size
    s = W.random_values((19, N), seed=3, dtype=np.float64)
    L = orc.Lattice(nx, n + 2, nz, 0.8, flags=flags)
    out = L.run(s, 2 * n, collide=False)
    fluid = flags == 0
    np.testing.assert_array_equal(out[:, fluid], s[:, fluid])
    # after n steps it is not the identity (the test is not vacuous)
    assert not np.array_equal(L.run(s, n, collide=False)[:, fluid], s[:, fluid])


def test_stream_only_is_permutation_with_obstacles(orc):
    nx, ny, nz = 9, 7, 6
    N = nx * ny * nz
    flags = W.random_flags(N, seed=4, solid_fraction=0.25)
    s = W.random_values((19, N), seed=5, dtype=np.float64)
    L = orc.Lattice(nx, ny, nz, 0.8, flags=flags)
    out = L.step(s, collide=False)
    fluid = flags == 0
    np.testing.assert_array_equal(np.sort(out[:, fluid].ravel()), np.sort(s[:, fluid].ravel()))


def test_rest_state_is_fixed_point(orc):
    nx, ny, nz = 8, 6, 5
    flags = W.random_flags(nx * ny * nz, seed=6, solid_fraction=0.2)
    L = orc.Lattice(nx, ny, nz, 0.7, flags=flags)
    s = _rest(orc, L.N)
    out = L.run(s, 10)
    fl = flags == 0
    np.testing.assert_allclose(out[:, fl], s[:, fl], rtol=0, atol=1e-16)


def _random_state(orc, N, seed, umax=0.05):
    return orc.init_equilibrium(N, W.random_density(N, seed, 0.02),
                                W.random_velocity(N, seed + 100, umax))


def test_mass_conserved_in_cavity_with_lid(orc):
    nx, ny, nz = 10, 9, 8
    flags = W.cavity_flags(nx, ny, nz)
    L = orc.Lattice(nx, ny, nz, 0.6, flags=flags, uw=(0.1, 0, 0))
    s = _random_state(orc, L.N, 7)
    fl = flags == 0
    m0 = s[:, fl].sum()
    s = L.run(s, 40)
    assert s[:, fl].sum() == pytest.approx(m0, rel=1e-13)


def test_momentum_conserved_periodic(orc):
    E, _, _ = orc.tables()
    L = orc.Lattice(7, 6, 5, 0.9)
    s = _random_state(orc, L.N, 8)
    p0 = E.T.astype(float) @ s.sum(1)
    s = L.run(s, 30)
    p1 = E.T.astype(float) @ s.sum(1)
    np.testing.assert_allclose(p1, p0, rtol=0, atol=1e-13)


def test_uniform_force_adds_momentum_linearly(orc):
    """Guo forcing: each step adds exactly F to the momentum of every fluid
    cell, so total momentum = P0 + t N F (periodic box)."""
    E, _, _ = orc.tables()
    F = np.array([1e-5, -2e-5, 3e-6])
    L = orc.Lattice(6, 5, 4, 0.7, force=F)
    s = _random_state(orc, L.N, 9, umax=0.01)
    p0 = E.T.astype(float) @ s.sum(1)
    t = 25
    s = L.run(s, t)
    p1 = E.T.astype(float) @ s.sum(1)
    np.testing.assert_allclose(p1, p0 + t * L.N * F, rtol=0, atol=1e-13)
    # the macroscopic velocity (with the -F/2 correction) grows at F/rho
    rho, u = L.macros(s)
    np.testing.assert_allclose(rho.sum() * 0 + (rho[None] * u).sum(1), p1 - L.N * F / 2,
                               rtol=0, atol=1e-13)


def _shear_rate(orc, n, tau, t1=200, t2=600, u0=1e-4):
    """Decay rate of u_x = u0 sin(2 pi y / n) in a 1 x n x 1 periodic box."""
    L = orc.Lattice(1, n, 1, tau)
    s = orc.init_equilibrium(L.N, None, W.shear_wave_velocity(1, n, 1, u0))
    y = np.arange(n)
    mode = np.sin(2 * np.pi * y / n)
    s = L.run(s, t1)
    a1 = L.macros(s)[1][0] @ mode
    s = L.run(s, t2 - t1)
    a2 = L.macros(s)[1][0] @ mode
    return np.log(a1 / a2) / (t2 - t1)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.2])
def test_shear_wave_viscosity(orc, tau):
    """Decay rate -> nu k^2 with nu = (tau - 1/2)/3; the relative error is
    O(k^2) (second-order method): below 1% at n = 32 and about 4x smaller at
    n = 64."""
    nu = (tau - 0.5) / 3
    errs = []
    for n in (32, 64):
        k = 2 * np.pi / n
        scale = (n / 32) ** 2
        rate = _shear_rate(orc, n, tau, t1=int(100 * scale), t2=int(400 * scale))
        errs.append(abs(rate / (nu * k * k) - 1))
    assert errs[0] < 0.01
    assert errs[1] < errs[0] / 3.0 or errs[1] < 1e-5


def test_taylor_green_3d_decay(orc):
    """The 32^3 Taylor-Green workload (tau 0.8, u0 0.05): the fundamental mode
    amplitude decays as exp(-3 nu k^2 t) to leading order."""
    n, tau, u0 = 32, 0.8, 0.05
    L = orc.Lattice(n, n, n, tau)
    u_init = W.taylor_green_velocity(n, n, n, u0)
    s = orc.init_equilibrium(L.N, None, u_init)
    mode = u_init[0] / u0
    nu = (tau - 0.5) / 3
    k = 2 * np.pi / n
    t = 100
    s = L.run(s, t)
    a = (L.macros(s)[1][0] @ mode) / (mode @ mode)
    expect = u0 * np.exp(-3 * nu * k * k * t)
    assert a == pytest.approx(expect, rel=0.03)


@pytest.mark.parametrize("tau", [0.6, 1.0, 0.5 + np.sqrt(3) / 4, 1.5])
def test_poiseuille_exact_discrete_profile(orc, tau):
    """Force-driven plane channel (fluid rows y = 1..n, walls at 0 and n+1).
    The steady BGK solution with halfway bounce-back is the parabola
    u(y) = F/(2 nu) (y - 1/2)(n + 1/2 - y) plus the bounce-back slip
    F (16 (tau - 1/2)^2 - 3) / (24 nu), which vanishes at
    tau = 1/2 + sqrt(3)/4 (Ginzburg & d'Humieres' result for bounce-back
    with a second-order force)."""
    n, F = 8, 1e-5
    L = orc.Lattice(1, n + 2, 1, tau, flags=W.channel_flags(n), force=(F, 0, 0))
    s = L.run(_rest(orc, L.N), 20000)
    ux = L.macros(s)[1][0][1:n + 1]
    nu = (tau - 0.5) / 3
    y = np.arange(1, n + 1)
    ref = F / (2 * nu) * (y - 0.5) * (n + 0.5 - y) + F / nu * (16 * (tau - 0.5) ** 2 - 3) / 24
    np.testing.assert_allclose(ux, ref, rtol=1e-10, atol=0)


@pytest.mark.parametrize("tau", [0.6, 1.1])
def test_couette_exact_linear_profile(orc, tau):
    """Lid moving at U on the wall at y = n+1 (moving-wall bounce-back with
    6 w_i rho_w e_i.u_w), resting wall at y = 0: u(y) = U (y - 1/2)/n exactly."""
    n, U = 8, 0.02
    flags = W.channel_flags(n, lid=True)
    L = orc.Lattice(1, n + 2, 1, tau, flags=flags, uw=(U, 0, 0))
    s = L.run(_rest(orc, L.N), 20000)
    ux = L.macros(s)[1][0][1:n + 1]
    y = np.arange(1, n + 1)
    np.testing.assert_allclose(ux, U * (y - 0.5) / n, rtol=1e-10, atol=0)


def test_macros_match_in_step_velocity(orc):
    """Reading u from the post-collision state with -F/2 gives the velocity
    used inside the collision, (m + F/2)/rho of the pre-collision state."""
    E, _, _ = orc.tables()
    F = np.array([2e-4, 0, -1e-4])
    L = orc.Lattice(4, 4, 4, 0.7, force=F)
    s0 = _random_state(orc, L.N, 10)
    s1 = L.step(s0)
    rho1, u1 = L.macros(s1)
    p = L.step(s0, collide=False)  # pre-collision (periodic: pure streaming)
    rho_p = p.sum(0)
    u_p = (E.T.astype(float) @ p + F[:, None] / 2) / rho_p
    np.testing.assert_allclose(rho1, rho_p, rtol=1e-14)
    np.testing.assert_allclose(u1, u_p, rtol=0, atol=1e-15)
