"""Pins of the oracle's lattice tables, equilibrium, collision and rounding.

Each test checks the oracle against something other than itself: the tables
printed in the paper (Eq. (4) and the weights after Eq. (5)), moment
identities that the equilibrium and the BGK collision must satisfy, and
library conversions for the storage rounding.
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_velocity_set_matches_eq4(orc):
    E, _, _ = orc.tables()
    printed = np.array(_golden("d3q19_velocities_eq4.txt"), dtype=np.int64)
    assert printed.shape == (3, 19)
    np.testing.assert_array_equal(E.T, printed)


def test_weights_match_text(orc):
    _, W, _ = orc.tables()
    for i, num, den in _golden("d3q19_weights.txt"):
        assert W[int(i)] == pytest.approx(int(num) / int(den), rel=0, abs=1e-17)


def test_opposites_and_isotropy(orc):
    E, W, OPP = orc.tables()
    # opposite pairs are (1,2), (3,4), ..., (17,18); rest maps to itself
    for i in range(19):
        np.testing.assert_array_equal(E[OPP[i]], -E[i])
        assert OPP[OPP[i]] == i
    assert OPP[0] == 0
    assert [OPP[i] for i in range(1, 19)] == [i + 1 if i % 2 else i - 1 for i in range(1, 19)]
    # distinct velocities, the full D3Q19 stencil: |e|^2 in {0, 1, 2}
    assert len({tuple(e) for e in E}) == 19
    assert sorted((E * E).sum(1).tolist()) == [0] + [1] * 6 + [2] * 12
    # lattice tensor identities: sum w = 1, odd moments vanish,
    # sum w e_a e_b = delta/3, sum w e_a e_b e_c e_d = (dd + dd + dd)/9
    assert W.sum() == pytest.approx(1.0, abs=1e-15)
    Ef = E.astype(float)
    np.testing.assert_allclose(np.einsum("i,ia->a", W, Ef), 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", W, Ef, Ef), np.eye(3) / 3, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", W, Ef, Ef, Ef), 0, atol=1e-16)
    d = np.eye(3)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", W, Ef, Ef, Ef, Ef), iso4,
                               atol=1e-16)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments(orc, seed):
    """Eq. (5) must reproduce rho (Eq. (6)), rho u (Eq. (7)) and the Euler
    stress rho/3 delta + rho u u."""
    E, _, _ = orc.tables()
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.8, 1.2)
    u = rng.uniform(-0.1, 0.1, 3)
    feq = orc.equilibrium(rho, u)
    Ef = E.astype(float)
    assert feq.sum() == pytest.approx(rho, rel=1e-14)
    np.testing.assert_allclose(Ef.T @ feq, rho * u, rtol=0, atol=1e-15)
    Pi = np.einsum("i,ia,ib->ab", feq, Ef, Ef)
    np.testing.assert_allclose(Pi, rho * np.eye(3) / 3 + rho * np.outer(u, u), atol=1e-15)
    # at rest the equilibrium is rho * w
    _, W, _ = orc.tables()
    np.testing.assert_allclose(orc.equilibrium(rho, np.zeros(3)), rho * W, rtol=1e-15)


def _moments(E, f):
    Ef = E.astype(float)
    return f.sum(), Ef.T @ f, np.einsum("i,ia,ib->ab", f, Ef, Ef)


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.0, 1.7])
@pytest.mark.parametrize("with_force", [False, True])
def test_collision_moment_relaxation(orc, tau, with_force):
    """BGK with the Guo force in moment space: mass is kept, momentum gains
    exactly F, and the second moment relaxes towards the Euler stress at rate
    1/tau with the Guo source (1 - 1/(2 tau)) (u F + F u)."""
    E, W, _ = orc.tables()
    rng = np.random.default_rng(int(tau * 100) + with_force)
    p = W * (1.0 + rng.uniform(-0.2, 0.2, 19))
    F = rng.uniform(-1e-3, 1e-3, 3) if with_force else np.zeros(3)
    s = orc.collide_cell(p, F, tau)
    rho0, m0, Pi0 = _moments(E, p)
    rho1, m1, Pi1 = _moments(E, s)
    assert rho1 == pytest.approx(rho0, rel=1e-14)
    np.testing.assert_allclose(m1, m0 + F, rtol=0, atol=1e-15)
    u = (m0 + F / 2) / rho0
    Pieq = rho0 * np.eye(3) / 3 + rho0 * np.outer(u, u)
    om = 1.0 / tau
    expect = (1 - om) * Pi0 + om * Pieq + (1 - om / 2) * (np.outer(u, F) + np.outer(F, u))
    np.testing.assert_allclose(Pi1, expect, rtol=0, atol=1e-15)


def test_collision_tau_one_lands_on_equilibrium(orc):
    """At tau = 1 without force the collision returns f^eq(rho, u) exactly,
    which is then a fixed point of collision at any tau."""
    _, W, _ = orc.tables()
    rng = np.random.default_rng(7)
    p = W * (1.0 + rng.uniform(-0.2, 0.2, 19))
    s = orc.collide_cell(p, None, 1.0)
    for tau in (0.6, 0.9, 1.4):
        np.testing.assert_allclose(orc.collide_cell(s, None, tau), s, rtol=0, atol=1e-15)


@pytest.mark.parametrize("tau", [0.6, 1.3])
def test_collision_jacobian_matches_central_differences(orc, tau):
    _, W, _ = orc.tables()
    rng = np.random.default_rng(11)
    p = W * (1.0 + rng.uniform(-0.1, 0.1, 19))
    F = rng.uniform(-1e-2, 1e-2, 3)
    J, dF, dtau = orc.collide_jacobian(p, F, tau)
    h = 1e-6
    Jfd = np.empty((19, 19))
    for j in range(19):
        e = np.zeros(19)
        e[j] = h
        Jfd[:, j] = (orc.collide_cell(p + e, F, tau) - orc.collide_cell(p - e, F, tau)) / (2 * h)
    np.testing.assert_allclose(J, Jfd, rtol=0, atol=2e-9)
    dFfd = np.empty((19, 3))
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        dFfd[:, b] = (orc.collide_cell(p, F + e, tau) - orc.collide_cell(p, F - e, tau)) / (2 * h)
    np.testing.assert_allclose(dF, dFfd, rtol=0, atol=2e-9)
    ht = 1e-6
    dtfd = (orc.collide_cell(p, F, tau + ht) - orc.collide_cell(p, F, tau - ht)) / (2 * ht)
    np.testing.assert_allclose(dtau, dtfd, rtol=0, atol=2e-9)


def test_round_half_matches_numpy_binary16(orc):
    rng = np.random.default_rng(3)
    vals = np.concatenate([
        rng.normal(0, 1e-2, 2000), rng.normal(0, 1e-5, 2000),   # normal and subnormal range
        rng.normal(0, 1e-7, 500), np.array([0.0, -0.0, 6.1e-5, 2.0 ** -24, 3 * 2.0 ** -25]),
    ])
    # exact ties: odd multiples of half a quantum
    ties = (2 * rng.integers(1, 1000, 200) + 1) * 2.0 ** -25
    vals = np.concatenate([vals, ties, -ties])
    got = np.array([orc.round_half(v) for v in vals])
    ref = vals.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(got, ref)


def test_round_bf16_matches_torch(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    f32 = np.concatenate([rng.normal(0, 1e-2, 3000), rng.normal(0, 1e-30, 200)]).astype(np.float32)
    # exact ties in float32: mantissa with the low 16 bits = 0x8000
    bits = rng.integers(0x3A000000, 0x3D000000, 300, dtype=np.int64) & ~0xFFFF | 0x8000
    f32 = np.concatenate([f32, bits.astype(np.uint32).view(np.float32)])
    got = np.array([orc.round_bf16(float(v)) for v in f32])
    ref = torch.from_numpy(f32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(got, ref)


def test_quantize_offsets(orc):
    _, W, _ = orc.tables()
    rng = np.random.default_rng(5)
    N = 64
    f = W[:, None] * (1 + rng.uniform(-0.3, 0.3, (19, N)))
    q16 = orc.quantize(f, "f16")
    ref16 = W[:, None] + (f - W[:, None]).astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(q16, ref16)
    q32 = orc.quantize(f, "f32")
    np.testing.assert_array_equal(q32, f.astype(np.float32).astype(np.float64))


def test_section_4_1_bounds_reproduce():
    """The throughput model of Section 4.1 (bytes per point over measured
    bandwidth) reproduces the printed MLUPS bounds with GB = 2^30 B."""
    for dev, bw, bpp, printed in _golden("theoretical_bounds_sec4_1.txt"):
        mlups = float(bw) * 2 ** 30 / int(bpp) / 1e6
        assert round(mlups) == int(printed), dev
