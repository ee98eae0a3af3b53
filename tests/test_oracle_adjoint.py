"""Pins of the oracle's discrete adjoint against central finite differences of
the oracle's own forward rollout (a different code path: the adjoint builds
explicit collision Jacobians and transposes streaming link by link).

Loss: L = (1/N_f) sum over fluid cells of |u(x, T) - u*(x)|^2, with u from the
post-collision state (Eqs. (6)-(7) with the Guo -F/2 correction).
"""
import numpy as np
import pytest

import workloads as W


def _setup(orc, geometry, seed, tau=0.7, uw=(0.0, 0.0, 0.0)):
    if geometry == "duct":
        nx, ny, nz = 6, 6, 5
        flags = W.duct_flags(nx, ny, nz)
    elif geometry == "cavity":
        nx, ny, nz = 6, 7, 5
        flags = W.cavity_flags(nx, ny, nz)
    else:
        nx, ny, nz = 5, 4, 4
        flags = W.random_flags(nx * ny * nz, seed, 0.2, moving_fraction=0.05)
    N = nx * ny * nz
    F = W.random_force_field(N, seed, 1e-3)
    Ft = W.random_force_field(N, seed + 1, 1e-3)
    s0 = orc.init_equilibrium(N, W.random_density(N, seed + 2, 0.01),
                              W.random_velocity(N, seed + 3, 0.02))
    return (nx, ny, nz), flags, F, Ft, s0, tau, uw


def _loss(orc, dims, flags, F, tau, uw, s0, T, ustar):
    L = orc.Lattice(*dims, tau, flags=flags, uw=uw, force_field=F)
    s = L.run(s0, T)
    _, u = L.macros(s)
    fl = flags == 0
    return ((u - ustar)[:, fl] ** 2).sum() / fl.sum(), u


def _target(orc, dims, flags, Ft, tau, uw, s0, T):
    L = orc.Lattice(*dims, tau, flags=flags, uw=uw, force_field=Ft)
    return L.macros(L.run(s0, T))[1]


@pytest.mark.parametrize("geometry,uw", [("duct", (0, 0, 0)), ("cavity", (0.05, 0, 0.02)),
                                         ("random", (0.03, -0.01, 0.0))])
def test_adjoint_matches_central_differences(orc, geometry, uw):
    dims, flags, F, Ft, s0, tau, _ = _setup(orc, geometry, seed=21)
    T = 12
    ustar = _target(orc, dims, flags, Ft, tau, uw, s0, T)
    L0, u = _loss(orc, dims, flags, F, tau, uw, s0, T, ustar)
    fl = flags == 0
    g = np.zeros_like(u)
    g[:, fl] = 2 * (u - ustar)[:, fl] / fl.sum()
    lat = orc.Lattice(*dims, tau, flags=flags, uw=uw, force_field=F)
    gF, gtau = lat.adjoint(s0, T, g)

    # d/dtau
    h = 1e-6 * tau
    Lp, _ = _loss(orc, dims, flags, F, tau + h, uw, s0, T, ustar)
    Lm, _ = _loss(orc, dims, flags, F, tau - h, uw, s0, T, ustar)
    fd_tau = (Lp - Lm) / (2 * h)
    assert gtau == pytest.approx(fd_tau, rel=1e-6)

    # directional derivatives along random force perturbations
    rng = np.random.default_rng(5)
    scale = 1e-3
    for _ in range(3):
        v = rng.normal(size=F.shape)
        h = 1e-4 * scale
        Lp, _ = _loss(orc, dims, flags, F + h * v, tau, uw, s0, T, ustar)
        Lm, _ = _loss(orc, dims, flags, F - h * v, tau, uw, s0, T, ustar)
        fd = (Lp - Lm) / (2 * h)
        assert (gF * v).sum() == pytest.approx(fd, rel=1e-6)

    # single cells and components (including a cell next to a wall)
    fluid_idx = np.flatnonzero(fl)
    for c in (fluid_idx[0], fluid_idx[len(fluid_idx) // 2], fluid_idx[-1]):
        for a in range(3):
            e = np.zeros_like(F)
            e[a, c] = 1.0
            h = 1e-7
            Lp, _ = _loss(orc, dims, flags, F + h * e, tau, uw, s0, T, ustar)
            Lm, _ = _loss(orc, dims, flags, F - h * e, tau, uw, s0, T, ustar)
            fd = (Lp - Lm) / (2 * h)
            assert gF[a, c] == pytest.approx(fd, rel=1e-5, abs=1e-12 * abs(gF).max())

    # solid cells carry no force gradient
    assert np.all(gF[:, ~fl] == 0)


def test_adjoint_zero_steps_is_direct_term(orc):
    """T = 0: only the direct dependence of u = (m - F/2)/rho on F remains."""
    dims, flags, F, _, s0, tau, uw = _setup(orc, "duct", seed=3)
    lat = orc.Lattice(*dims, tau, flags=flags, force_field=F)
    rho, _ = lat.macros(s0)
    g = W.random_velocity(flags.size, 9, 1.0)
    g[:, flags != 0] = 0
    gF, gtau = lat.adjoint(s0, 0, g)
    fl = flags == 0
    np.testing.assert_allclose(gF[:, fl], -g[:, fl] / (2 * rho[fl]), rtol=1e-15)
    assert gtau == 0.0
