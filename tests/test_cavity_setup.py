"""Host-side pieces of the cavity validation workload (Section 5): the
geometry, the Eq. (8) scaling and the resolution comparison."""
import numpy as np
import pytest

import workloads as W
from paper_1309_1983_amd import cavity


@pytest.mark.parametrize("L", [2, 8, 16, 18])
def test_cavity_geometry_is_the_onsite_cavity(L):
    n = L + 3
    nx, ny, nz = cavity.box_shape(L)
    assert nx % 4 == 0 and nx - n < 4 and ny == nz == n
    f = cavity.cavity_flags(L).reshape(n, n, nx)
    ref = W.onsite_cavity_flags(n, n, n).reshape(n, n, n)
    np.testing.assert_array_equal(f[:, :, :n], ref)
    assert np.all(f[:, :, n:] == W.WALL)                         # padding along x is solid
    assert np.all(f[1:-1, L + 1, 1:n - 1] == W.ONSITE_MOVING)   # the lid, edges included
    assert np.count_nonzero(f == W.ONSITE) + np.count_nonzero(f == W.ONSITE_MOVING) \
        == (L + 1) ** 3 - (L - 1) ** 3


def test_odd_side_is_rejected():
    with pytest.raises(ValueError):
        cavity.cavity_flags(15)


@pytest.mark.parametrize("Re,L,u", [(100, 64, 0.1), (400, 128, 0.05), (1000, 256, 0.1)])
def test_eq8_scaling(Re, L, u):
    tau = cavity.tau_for(Re, L, u)
    assert u == pytest.approx((tau - 0.5) * Re / (3 * L), rel=1e-14)
    assert cavity.lid_speed_for(Re, L, tau) == pytest.approx(u, rel=1e-14)
    nu = (tau - 0.5) / 3
    assert u * L / nu == pytest.approx(Re, rel=1e-12)


def _result(L, ux, uy):
    pos = np.arange(L + 1) / L
    return cavity.CavityResult(Re=100, L=L, tau=0.6, u_lid=0.1, steps=1, converged=True, residual=0.0,
                               finite=True, y=pos, ux=ux, x=pos, uy=uy, seconds=1.0, glups=1.0)


def test_resolution_differences_recover_the_order_of_a_known_error():
    # profiles = exact + C h^2 on each grid: differences shrink 4x per doubling
    exact = lambda s: np.sin(np.pi * s)
    res = []
    for L in (8, 16, 32):
        s = np.arange(L + 1) / L
        res.append(_result(L, exact(s) + 0.3 * (1.0 / L) ** 2 * np.cos(s), exact(s)))
    diffs, orders = cavity.resolution_differences(res)
    assert diffs[0] > diffs[1] > 0
    assert orders[0] == pytest.approx(2.0, abs=1e-9)


def test_common_nodes_of_a_three_to_two_refinement():
    ia, ib = cavity.common_nodes(8, 12)
    np.testing.assert_array_equal(ia, [0, 2, 4, 6, 8])
    np.testing.assert_array_equal(ib, [0, 3, 6, 9, 12])
    np.testing.assert_allclose(ia / 8, ib / 12, rtol=0, atol=0)
    ia, ib = cavity.common_nodes(16, 32)
    np.testing.assert_array_equal(ia, np.arange(17))
    np.testing.assert_array_equal(ib, 2 * np.arange(17))


def test_resolution_differences_at_a_three_to_two_refinement():
    # exact + C h^2 on grids of side 8, 12, 18: the differences at the shared
    # positions are C (h_a^2 - h_b^2) cos(s) and give order 2 at ratio 3/2
    exact = lambda s: np.sin(np.pi * s)
    res = []
    for L in (8, 12, 18):
        s = np.arange(L + 1) / L
        res.append(_result(L, exact(s), exact(s) + 0.3 * (1.0 / L) ** 2 * np.cos(s)))
    diffs, orders = cavity.resolution_differences(res)
    assert diffs[0] == pytest.approx(0.3 * (1 / 64 - 1 / 144), rel=1e-12)
    assert orders[0] == pytest.approx(2.0, abs=1e-9)
    with pytest.raises(ValueError):
        cavity.resolution_differences([res[0], res[0]])
