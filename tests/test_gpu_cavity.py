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
