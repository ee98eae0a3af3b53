"""GPU parity of the on-site velocity nodes (flags 3 and 4; the boundary type
of the paper's cavity validation, Section 5) against the FP64 oracle, which
solves each node's mass and momentum conditions as a 4x4 linear system while
the kernels use the closed form.

- FP32: max |df|/|f| <= 1e-5 over all fluid and on-site points after 100
  steps, through the one-point kernel (ragged nx) and the vector kernel, with
  a lid velocity along all three axes, uniform and per-point forces;
- the AA and AB patterns agree bit for bit, and so do the vector and
  one-point kernels;
- every on-site node reports its prescribed velocity;
- 16-bit storage: one step equals the oracle's step followed by the same
  offset rounding, to one unit of the format;
- nodes whose solid neighbours are not a box face, edge or corner are
  rejected at creation; the adjoint refuses lattices with on-site nodes;
- 128^3 cavity in the benchmark's launch configuration: full-domain parity
  after 100 steps.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import near_rest_state, oracle_lattice

pytestmark = pytest.mark.gpu

Q = 19
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1309_1983_amd
    paper_1309_1983_amd.lib()


def _fluid(flags):
    return (flags != W.WALL) & (flags != W.MOVING_WALL)


def _rel_err(got, ref, flags):
    fl = _fluid(flags)
    return float(np.max(np.abs(got[:, fl].astype(np.float64) - ref[:, fl]) / np.abs(ref[:, fl])))


def _run(shape, tau, flags, s0, steps, uw=None, force=None, ff=None, **kw):
    from paper_1309_1983_amd import Lattice
    lat = Lattice(*shape, tau, flags=flags, **kw)
    if uw is not None:
        lat.set_wall_velocity(*uw)
    if force is not None:
        lat.set_force(force)
    if ff is not None:
        lat.set_force(torch.from_numpy(ff))
    lat.set_populations(torch.from_numpy(s0))
    lat.step(steps)
    out = lat.populations().cpu().numpy()
    _, u = lat.macros()
    lat.close()
    return out, u.cpu().numpy()


CASES = {
    # name: (shape, tau, lid velocity, uniform force, per-point force amplitude)
    "ragged_one_point": ((13, 11, 10), 0.7, (0.05, 0.01, -0.02), None, 1e-4),
    "vector": ((16, 12, 10), 0.65, (0.08, 0.0, 0.0), (1e-5, -2e-5, 5e-6), None),
    "vector_field": ((24, 9, 7), 0.9, (0.03, -0.02, 0.04), None, 1e-4),
    # 65 four-point groups per row: the vector step's one-dimensional grid
    "flat_rows": ((260, 7, 6), 0.7, (0.05, 0.0, 0.01), (2e-5, 0.0, 0.0), None),
}


def _case(name):
    shape, tau, uw, force, famp = CASES[name]
    flags = W.onsite_cavity_flags(*shape)
    N = flags.size
    ff = None if famp is None else W.random_force_field(N, 7, famp).astype(np.float32)
    s0 = near_rest_state(N, 8)
    return shape, tau, flags, uw, force, ff, s0


@pytest.mark.parametrize("name", list(CASES))
def test_onsite_f32_matches_oracle_after_100_steps(name):
    shape, tau, flags, uw, force, ff, s0 = _case(name)
    got, u = _run(shape, tau, flags, s0, 100, uw=uw, force=force, ff=ff)
    olat = oracle_lattice(shape, tau, flags=flags, uw=uw, force=force, force_field=ff)
    ref = olat.run(s0.astype(np.float64), 100)
    err = _rel_err(got, ref, flags)
    print(f"on-site {name}: max rel |df| after 100 steps = {err:.3e}")
    assert err <= TOL
    uw32 = np.asarray(uw, np.float32).astype(np.float64)
    assert np.max(np.abs(u[:, flags == W.ONSITE])) <= 2e-6
    assert np.max(np.abs(u[:, flags == W.ONSITE_MOVING] - uw32[:, None])) <= 2e-6


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_onsite_aa_equals_ab_and_vector_equals_one_point(storage):
    shape, tau, flags, uw, force, ff, s0 = _case("vector_field")
    fl = _fluid(flags)
    for steps in (1, 4, 5):
        ab, _ = _run(shape, tau, flags, s0, steps, uw=uw, ff=ff, storage=storage)
        aa, _ = _run(shape, tau, flags, s0, steps, uw=uw, ff=ff, storage=storage, pattern="aa")
        one, _ = _run(shape, tau, flags, s0, steps, uw=uw, ff=ff, storage=storage, cells_per_lane=1)
        np.testing.assert_array_equal(aa[:, fl], ab[:, fl], err_msg=f"AA {storage} {steps}")
        np.testing.assert_array_equal(one[:, fl], ab[:, fl], err_msg=f"one-point {storage} {steps}")
        if storage != "f32":
            v8, _ = _run(shape, tau, flags, s0, steps, uw=uw, ff=ff, storage=storage, cells_per_lane=8) \
                if shape[0] % 8 == 0 else (ab, None)
            np.testing.assert_array_equal(v8[:, fl], ab[:, fl], err_msg=f"width 8 {storage} {steps}")


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_onsite_16bit_one_step_matches_rounded_oracle(storage):
    shape, tau = (24, 10, 9), 0.7
    flags = W.onsite_cavity_flags(*shape)
    N = flags.size
    _, Wt, _ = oracle.tables()
    s0 = near_rest_state(N, 9)
    q = oracle.quantize(s0.astype(np.float64), storage)      # representable start
    plain = q.astype(np.float32)
    uw, force = (0.05, 0.0, 0.02), (1e-5, 0.0, -1e-5)
    got, _ = _run(shape, tau, flags, plain, 1, uw=uw, force=force, storage=storage)
    olat = oracle_lattice(shape, tau, flags=flags, uw=uw, force=force)
    ref_q = oracle.quantize(olat.step(plain.astype(np.float64)), storage)
    fl = _fluid(flags)
    hq = np.abs(ref_q - Wt[:, None])[:, fl]
    mant = 10 if storage == "f16" else 7
    emin = -14 if storage == "f16" else -126
    ulp = 2.0 ** (np.maximum(np.floor(np.log2(np.maximum(hq, 1e-300))), emin) - mant)
    diff = np.abs(got[:, fl].astype(np.float64) - ref_q[:, fl])
    rep = 4e-8
    assert np.all(diff <= ulp * 1.01 + rep), float(np.max((diff - rep) / ulp))


def test_onsite_channel_reaches_the_exact_poiseuille_profile():
    """Steady plane Poiseuille flow between on-site walls on the GPU: the
    parabola with zero velocity on the node planes. With FP32 storage of the
    populations the approach to the steady state stalls once the per-step
    correction drops below the storage resolution (about 1e-6 in velocity),
    so the force is chosen to keep that well under the tolerance."""
    h, tau, F = 16, 0.8, 1e-4
    nu = (tau - 0.5) / 3
    flags = W.onsite_channel_flags(h, nx=8, nz=4)
    shape = (8, h + 3, 4)
    N = flags.size
    s0 = oracle.init_equilibrium(N).astype(np.float32)
    _, u = _run(shape, tau, flags, s0, int(30 * h * h / nu), force=(F, 0, 0))
    sy = np.arange(h + 3) - 1.0
    exact = F * sy * (h - sy) / (2 * nu)
    ux = u[0].reshape(4, h + 3, 8)[:, 1:-1, :]
    err = np.max(np.abs(ux - exact[None, 1:-1, None])) / exact.max()
    print(f"on-site Poiseuille h={h}: max rel error {err:.2e}")
    assert err <= 2e-4
    assert np.max(np.abs(u[1:])) <= 1e-6


def test_invalid_onsite_neighbourhoods_are_rejected():
    from paper_1309_1983_amd import LBMError, Lattice
    shape = (8, 8, 8)
    N = 512
    lone = np.zeros(N, np.uint8)
    lone[(4 * 8 + 4) * 8 + 4] = W.ONSITE              # no solid neighbour
    diag = np.zeros(N, np.uint8)
    diag[(4 * 8 + 4) * 8 + 4] = W.ONSITE
    diag[(5 * 8 + 5) * 8 + 4] = W.WALL                # one diagonal solid neighbour
    slab = np.zeros(N, np.uint8).reshape(8, 8, 8)
    slab[:, 3, :] = W.ONSITE
    slab[:, 2, :] = W.WALL
    slab[:, 4, :] = W.WALL                            # solid on both sides along y
    for name, fl in (("lone", lone), ("diagonal", diag), ("slab", slab.reshape(-1))):
        with pytest.raises(LBMError, match="INVALID"):
            Lattice(*shape, 0.7, flags=fl)
    ok = Lattice(*shape, 0.7, flags=W.onsite_cavity_flags(*shape))
    ok.close()


def test_adjoint_refuses_onsite_nodes():
    from paper_1309_1983_amd import LBMError, Lattice
    shape = (8, 8, 8)
    lat = Lattice(*shape, 0.7, flags=W.onsite_cavity_flags(*shape))
    with pytest.raises(LBMError, match="STATE"):
        lat.forward_checkpointed(4, 2)
    lat.close()


@pytest.mark.timeout(300)
def test_onsite_cavity128_full_domain_100_steps():
    """128^3 on-site cavity (lid 0.1 along +x, tau 0.6) in the default
    launch configuration, every point after 100 steps from a random
    near-rest state."""
    n, tau, lid = 128, 0.6, 0.1
    flags = W.onsite_cavity_flags(n, n, n)
    s0 = near_rest_state(flags.size, 19)
    got, u = _run((n, n, n), tau, flags, s0, 100, uw=(lid, 0, 0))
    olat = oracle_lattice((n, n, n), tau, flags=flags, uw=(lid, 0, 0))
    ref = olat.run(s0.astype(np.float64), 100)
    err = _rel_err(got, ref, flags)
    print(f"on-site cavity 128^3, 100 steps: max rel |df| = {err:.3e}")
    assert err <= TOL
    assert np.max(np.abs(u[0, flags == W.ONSITE_MOVING] - np.float32(lid))) <= 2e-6
