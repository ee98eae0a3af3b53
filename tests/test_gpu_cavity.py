"""The cavity validation workload (Section 5) on the GPU: steady centreline
profiles of the on-site-walled cavity against the FP64 oracle run for the
same number of steps, and convergence between doubled resolutions (the
reference profiles the paper compares with are not available, so the
resolution study is what the workload can show; parity unpinned beyond
that)."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_common import oracle_lattice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1309_1983_amd
    paper_1309_1983_amd.lib()


def test_steady_cavity_matches_oracle():
    from paper_1309_1983_amd import cavity
    Re, L, u = 20, 16, 0.05
    r = cavity.run(Re, L, u_lid=u, tol=1e-6, check_every=100)
    assert r.converged and r.finite
    nx, n, _ = cavity.box_shape(L)
    flags = cavity.cavity_flags(L)
    olat = oracle_lattice((nx, n, n), np.float32(r.tau), flags=flags, uw=(u, 0, 0))
    s = olat.run(oracle.init_equilibrium(nx * n * n), r.steps)
    _, uo = olat.macros(s)
    uo = uo.reshape(3, n, n, nx)
    m = 1 + L // 2
    ux = uo[0, m, 1:L + 2, m] / np.float32(u)
    uy = uo[1, m, m, 1:L + 2] / np.float32(u)
    err = max(np.max(np.abs(r.ux - ux)), np.max(np.abs(r.uy - uy)))
    print(f"Re {Re} L {L}: {r.steps} steps, centreline |u_gpu - u_oracle| / u_lid = {err:.2e}")
    assert err <= 1e-4
    # the lid row and the resting walls carry their prescribed velocities
    assert r.ux[-1] == pytest.approx(1.0, abs=1e-5) and abs(r.ux[0]) <= 1e-5


def test_cavity_profiles_converge_with_resolution():
    """Re 20 with tau fixed (diffusive scaling: the lid speed halves with
    each doubling of L). The lid's corners are singular (the lid velocity
    jumps to zero at the side walls), which caps the observed order near one;
    the differences must shrink by at least that."""
    from paper_1309_1983_amd import cavity
    res = [cavity.run(20, L, tau=0.62, tol=1e-5, check_every=1000) for L in (16, 32, 64)]
    assert all(r.converged and r.finite for r in res)
    diffs, orders = cavity.resolution_differences(res)
    rms, rms_orders = cavity.resolution_differences(res, "rms")
    print(f"Re 20: max profile differences {diffs} (order {orders}); RMS {rms} (order {rms_orders})")
    assert diffs[1] < diffs[0] / 1.8 and rms[1] < rms[0] / 1.8


def _oracle_profiles(r, L):
    from paper_1309_1983_amd import cavity
    nx, n, _ = cavity.box_shape(L)
    olat = oracle_lattice((nx, n, n), np.float32(r.tau), flags=cavity.cavity_flags(L),
                          uw=(np.float32(r.u_lid), 0, 0))
    s = olat.run(oracle.init_equilibrium(nx * n * n), r.steps)
    _, uo = olat.macros(s)
    uo = uo.reshape(3, n, n, nx)
    m = 1 + L // 2
    return uo[0, m, 1:L + 2, m] / np.float32(r.u_lid), uo[1, m, m, 1:L + 2] / np.float32(r.u_lid)


@pytest.mark.timeout(300)
def test_re100_cavity_matches_oracle():
    """Re 100, the paper's lowest validation Reynolds number (Section 5), at
    L = 32 with tau 0.6 (Eq. (8): lid speed 0.104), run from rest to a steady
    state on the GPU; the oracle runs the same number of steps in FP64."""
    from paper_1309_1983_amd import cavity
    L = 32
    r = cavity.run(100, L, tau=0.6, tol=1e-5)
    assert r.converged and r.finite
    ux, uy = _oracle_profiles(r, L)
    err = max(np.max(np.abs(r.ux - ux)), np.max(np.abs(r.uy - uy)))
    print(f"Re 100 L {L}: {r.steps} steps, centreline |u_gpu - u_oracle| / u_lid = {err:.2e}; "
          f"min u_x/U {r.ux.min():.4f} at y/L {r.y[np.argmin(r.ux)]:.3f}")
    assert err <= 1e-4
    # the primary vortex: the vertical centreline's u_x reverses below the lid
    assert r.ux.min() < -0.1 and 0.3 < r.y[np.argmin(r.ux)] < 0.7


@pytest.mark.timeout(300)
def test_re100_profiles_converge_with_resolution():
    """Re 100 at L = 32, 64, 128 with tau 0.6 fixed (diffusive scaling). The
    lid's singular corners cap the observed order near one: each doubling
    must shrink the profile differences by at least 1.6."""
    from paper_1309_1983_amd import cavity
    res = [cavity.run(100, L, tau=0.6, tol=1e-5) for L in (32, 64, 128)]
    assert all(r.converged and r.finite for r in res)
    diffs, orders = cavity.resolution_differences(res)
    rms, rms_orders = cavity.resolution_differences(res, "rms")
    print(f"Re 100: steps {[r.steps for r in res]}; max profile differences {diffs} (order {orders}); "
          f"RMS {rms} (order {rms_orders})")
    assert diffs[1] < diffs[0] / 1.6 and rms[1] < rms[0] / 1.6
