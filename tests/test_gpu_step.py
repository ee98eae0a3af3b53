"""GPU parity of the forward step against the FP64 oracle (through the C ABI).

- streaming with bounce-back is an exact permutation: bit-exact vs the oracle
  (AB and AA, FP32 and 16-bit storage);
- FP32 steps: max |df|/|f| <= 1e-5 over fluid cells after 100 steps (the
  tolerance the method's target fixes), on ragged lattices that span
  several work-groups, every boundary kind, uniform and per-cell forces;
- AA and AB agree bit for bit (same storage); results do not depend on the
  work-group shape;
- 16-bit storage: one step equals the oracle's step followed by the same
  offset rounding to within one unit of the 16-bit format.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import f32, fluid_rel_err, near_rest_state, oracle_lattice

pytestmark = pytest.mark.gpu

Q = 19
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1309_1983_amd
    paper_1309_1983_amd.lib()


def _lattice(shape, tau, flags=None, uw=None, force=None, force_field=None, **kw):
    from paper_1309_1983_amd import Lattice
    lat = Lattice(*shape, tau, flags=flags, **kw)
    if uw is not None:
        lat.set_wall_velocity(*uw)
    if force is not None:
        lat.set_force(force)
    if force_field is not None:
        lat.set_force(torch.from_numpy(np.asarray(force_field, dtype=np.float32)))
    return lat


def _gpu_run(shape, tau, s0, steps, stream_only=False, **kw):
    lat = _lattice(shape, tau, **kw)
    lat.set_populations(torch.from_numpy(s0))
    if stream_only:
        lat.stream_only(steps)
    else:
        lat.step(steps)
    out = lat.populations().cpu().numpy()
    lat.close()
    return out


# ----------------------------- streaming -----------------------------------

STREAM_CASES = [
    ((37, 23, 19), 0.25, 0.05),
    ((64, 8, 5), 0.10, 0.0),
    ((1, 7, 3), 0.20, 0.05),      # degenerate widths: x neighbours wrap onto the cell itself
    ((130, 3, 2), 0.0, 0.0),      # periodic only, ragged tail over two work-groups
]


@pytest.mark.parametrize("pattern", ["ab", "aa"])
@pytest.mark.parametrize("shape,solid,moving", STREAM_CASES)
def test_stream_only_bit_exact_f32(pattern, shape, solid, moving):
    N = int(np.prod(shape))
    flags = W.random_flags(N, seed=N, solid_fraction=solid, moving_fraction=moving)
    s0 = W.random_values((Q, N), seed=N + 1, lo=-1.0, hi=1.0)
    olat = oracle.Lattice(*shape, 0.8, flags=flags)
    ref = s0.astype(np.float64)
    for steps in (1, 2, 3):
        ref = olat.step(ref, collide=False)
        got = _gpu_run(shape, 0.8, s0, steps, stream_only=True, flags=flags, pattern=pattern,
                       uw=(0.05, 0.0, 0.0))
        fl = flags == 0
        np.testing.assert_array_equal(got[:, fl], ref[:, fl].astype(np.float32), err_msg=f"step {steps}")


def _offset_state(N, seed, fmt):
    """Plain FP32 populations whose 16-bit offsets are exactly the random
    values h (|h| in [1e-4, 2e-3], random sign, representable in fmt)."""
    _, Wt, _ = oracle.tables()
    rng = np.random.default_rng(seed)
    h = rng.uniform(1e-4, 2e-3, (Q, N)) * rng.choice([-1.0, 1.0], (Q, N))
    h = np.array([[oracle.round_half(v) if fmt == "f16" else oracle.round_bf16(v) for v in row]
                  for row in h])
    plain = (Wt.astype(np.float32)[:, None] + h.astype(np.float32)).astype(np.float32)
    return h, plain


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("pattern", ["ab", "aa"])
def test_stream_only_bit_exact_16bit(storage, pattern):
    shape = (37, 11, 9)
    N = int(np.prod(shape))
    flags = W.random_flags(N, seed=3, solid_fraction=0.2, moving_fraction=0.05)
    h, plain = _offset_state(N, 4, storage)
    _, Wt, _ = oracle.tables()
    olat = oracle.Lattice(*shape, 0.8, flags=flags)
    ref_h = h
    fl = flags == 0
    for steps in (1, 2, 3):
        ref_h = olat.step(ref_h, collide=False)
        expect = (Wt.astype(np.float32)[:, None] + ref_h.astype(np.float32)).astype(np.float32)
        got = _gpu_run(shape, 0.8, plain, steps, stream_only=True, flags=flags, storage=storage,
                       pattern=pattern)
        np.testing.assert_array_equal(got[:, fl], expect[:, fl], err_msg=f"step {steps}")


# ----------------------------- FP32 steps ----------------------------------

def _case(name):
    """(shape, tau, flags, uw, force, force_field, s0) of the named workload."""
    if name == "tgv32":
        shape, tau = (32, 32, 32), 0.8
        N = 32 ** 3
        s0 = oracle.init_equilibrium(N, None, W.taylor_green_velocity(32, 32, 32, 0.05)).astype(np.float32)
        return shape, tau, None, None, None, None, s0
    if name == "cavity_ragged":
        shape, tau = (70, 37, 29), 0.6
        flags = W.cavity_flags(*shape)
        return shape, tau, flags, (0.1, 0, 0), None, None, near_rest_state(flags.size, 11)
    if name == "spheres_duct":
        shape, tau = (48, 40, 64), 0.7
        flags = W.sphere_duct_flags(*shape, seed=5, solid_fraction=0.10)
        return shape, tau, flags, None, (0, 0, 1e-6), None, near_rest_state(flags.size, 12, 0.005, 0.01)
    if name in ("random_walls_field", "random_walls_field_x4", "random_walls_wide_rows"):
        # wide rows: 65 four-point groups per row, the vector step's one-dimensional grid
        shape = {"random_walls_field": (33, 17, 11), "random_walls_field_x4": (36, 17, 11),
                 "random_walls_wide_rows": (260, 9, 7)}[name]
        tau = 0.9
        N = int(np.prod(shape))
        flags = W.random_flags(N, seed=13, solid_fraction=0.2, moving_fraction=0.05)
        ff = W.random_force_field(N, 14, 1e-4).astype(np.float32)
        return shape, tau, flags, (0.05, -0.02, 0.03), None, ff, near_rest_state(N, 15)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["tgv32", "cavity_ragged", "spheres_duct", "random_walls_field",
                                  "random_walls_field_x4", "random_walls_wide_rows"])
def test_f32_step_matches_oracle_after_100_steps(name):
    shape, tau, flags, uw, force, ff, s0 = _case(name)
    got = _gpu_run(shape, tau, s0, 100, flags=flags, uw=uw, force=force, force_field=ff)
    olat = oracle_lattice(shape, tau, flags=flags, uw=uw if uw else (0, 0, 0), force=force,
                          force_field=ff)
    ref = olat.run(s0.astype(np.float64), 100)
    err = fluid_rel_err(got.astype(np.float64), ref, flags)
    print(f"{name}: max rel |df| after 100 steps = {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("name,pattern", [("random_walls_field", "ab"), ("random_walls_field_x4", "ab"),
                                          ("spheres_duct", "ab"), ("random_walls_field_x4", "aa"),
                                          ("random_walls_wide_rows", "ab")])
def test_fused_macros_match_separate_pass_and_oracle(name, pattern):
    """rho and u written by the step itself (168 B per point variant) equal the
    separate macroscopic pass over the resulting state to FP32 rounding, and
    the oracle's macros of its own run, and the populations are unchanged."""
    shape, tau, flags, uw, force, ff, s0 = _case(name)
    lat = _lattice(shape, tau, flags=flags, uw=uw, force=force, force_field=ff, pattern=pattern)
    lat.set_populations(torch.from_numpy(s0))
    rho_f, u_f = (t.cpu().numpy().astype(np.float64) for t in lat.step_macros(20))
    rho_s, u_s = (t.cpu().numpy().astype(np.float64) for t in lat.macros())
    f_fused = lat.populations().cpu().numpy()
    lat.close()
    plain = _gpu_run(shape, tau, s0, 20, flags=flags, uw=uw, force=force, force_field=ff, pattern=pattern)
    fl = flags == 0
    np.testing.assert_array_equal(f_fused[:, fl], plain[:, fl])
    assert np.max(np.abs(rho_f - rho_s)[fl]) <= 4e-7
    assert np.max(np.abs(u_f - u_s)[:, fl]) <= 4e-7
    assert np.all(rho_f[~fl] == 0) and np.all(u_f[:, ~fl] == 0)
    olat = oracle_lattice(shape, tau, flags=flags, uw=uw if uw else (0, 0, 0), force=force,
                          force_field=ff)
    rho_ref, u_ref = olat.macros(olat.run(s0.astype(np.float64), 20))
    assert np.max(np.abs(rho_f - rho_ref)[fl]) <= 1e-6
    assert np.max(np.abs(u_f - u_ref)[:, fl]) <= 1e-6


def test_init_equilibrium_matches_oracle():
    shape, tau, flags, uw, force, ff, _ = _case("random_walls_field")
    N = int(np.prod(shape))
    rho0 = W.random_density(N, 21, 0.02).astype(np.float32)
    u0 = W.random_velocity(N, 22, 0.05).astype(np.float32)
    lat = _lattice(shape, tau, flags=flags)
    lat.init_equilibrium(torch.from_numpy(rho0), torch.from_numpy(u0))
    f_init = lat.populations().cpu().numpy().astype(np.float64)
    lat.close()
    ref_init = oracle.init_equilibrium(N, rho0.astype(np.float64), u0.astype(np.float64))
    assert np.max(np.abs(f_init - ref_init) / ref_init) <= 1e-6


@pytest.mark.parametrize("name", ["random_walls_field", "spheres_duct"])
def test_macros_match_oracle(name):
    """rho and u after 20 steps from the same initial state: GPU macros of the
    GPU run vs oracle macros of the oracle run."""
    shape, tau, flags, uw, force, ff, s0 = _case(name)
    lat = _lattice(shape, tau, flags=flags, uw=uw, force=force, force_field=ff)
    lat.set_populations(torch.from_numpy(s0))
    lat.step(20)
    rho, u = (t.cpu().numpy().astype(np.float64) for t in lat.macros())
    lat.close()
    olat = oracle_lattice(shape, tau, flags=flags, uw=uw if uw else (0, 0, 0), force=force,
                          force_field=ff)
    rho_ref, u_ref = olat.macros(olat.run(s0.astype(np.float64), 20))
    fl = flags == 0
    assert np.max(np.abs(rho - rho_ref)[fl]) <= 1e-6
    assert np.max(np.abs(u - u_ref)[:, fl]) <= 1e-6
    assert np.all(rho[~fl] == 0) and np.all(u[:, ~fl] == 0)


@pytest.mark.parametrize("name", ["random_walls_field", "random_walls_field_x4"])
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_aa_equals_ab_bitwise(storage, name):
    shape, tau, flags, uw, force, ff, s0 = _case(name)
    for steps in (1, 2, 5):
        a = _gpu_run(shape, tau, s0, steps, flags=flags, uw=uw, force_field=ff, storage=storage,
                     pattern="ab")
        b = _gpu_run(shape, tau, s0, steps, flags=flags, uw=uw, force_field=ff, storage=storage,
                     pattern="aa")
        fl = flags == 0
        np.testing.assert_array_equal(a[:, fl], b[:, fl], err_msg=f"{storage} after {steps}")


@pytest.mark.parametrize("block", [(32, 1), (64, 1), (100, 3), (128, 2), (256, 4), (16, 16), (70, 1)])
def test_block_shape_does_not_change_results(block):
    shape, tau, flags, uw, force, ff, s0 = _case("cavity_ragged")
    ref = _gpu_run(shape, tau, s0, 7, flags=flags, uw=uw)
    got = _gpu_run(shape, tau, s0, 7, flags=flags, uw=uw, block=block)
    np.testing.assert_array_equal(got, ref)


FOUR_CELL_CASES = [
    # (shape, solid fraction, moving fraction, uniform force, field)
    ((36, 17, 11), 0.2, 0.05, None, True),      # walls everywhere, per-point force
    ((64, 9, 7), 0.0, 0.0, (1e-5, -2e-5, 3e-6), False),   # periodic in x: row-end wrap
    ((4, 5, 6), 0.15, 0.05, None, False),       # one quad per row: both row ends in one work-item
    ((256, 3, 2), 0.3, 0.1, (0, 0, 1e-5), False),
    ((8, 6, 5), 0.1, 0.05, None, True),         # one 8-point group per row
    ((40, 7, 3), 0.0, 0.0, None, True),         # periodic in x, five 8-point groups per row
    ((260, 5, 3), 0.2, 0.05, None, True),       # 65 four-point groups per row: one-dimensional grid
    ((520, 3, 2), 0.1, 0.05, (1e-5, 0, 0), False),   # 65 eight-point groups per row
]


@pytest.mark.parametrize("storage,width", [("f32", 4), ("f16", 4), ("bf16", 4), ("f16", 8), ("bf16", 8)])
@pytest.mark.parametrize("case", range(len(FOUR_CELL_CASES)))
def test_vector_kernel_equals_one_point_kernel(storage, width, case):
    """The several-points-per-work-item AB kernel performs the same per-point
    arithmetic as the one-point kernel: fluid results agree bit for bit,
    including the periodic wrap at row ends and solid points inside a group."""
    shape, solid, moving, force, field = FOUR_CELL_CASES[case]
    if shape[0] % width:
        pytest.skip(f"nx = {shape[0]} is not a multiple of {width}")
    N = int(np.prod(shape))
    flags = W.random_flags(N, seed=40 + case, solid_fraction=solid, moving_fraction=moving)
    ff = W.random_force_field(N, 41, 1e-4).astype(np.float32) if field else None
    s0 = near_rest_state(N, 42 + case)
    kw = dict(flags=flags, uw=(0.05, -0.02, 0.03), force=force, force_field=ff, storage=storage)
    for steps in (1, 3):
        one = _gpu_run(shape, 0.8, s0, steps, cells_per_lane=1, **kw)
        vec = _gpu_run(shape, 0.8, s0, steps, cells_per_lane=width, **kw)
        fl = flags == 0
        np.testing.assert_array_equal(vec[:, fl], one[:, fl], err_msg=f"{storage} {shape} {steps}")
    stream1 = _gpu_run(shape, 0.8, s0, 2, stream_only=True, cells_per_lane=1, **kw)
    streamv = _gpu_run(shape, 0.8, s0, 2, stream_only=True, cells_per_lane=width, **kw)
    np.testing.assert_array_equal(streamv[:, flags == 0], stream1[:, flags == 0])


@pytest.mark.parametrize("block", [(8, 1), (16, 4), (64, 4), (64, 1), (32, 8), (3, 5)])
def test_four_cell_block_shapes(block):
    shape, tau, flags, uw, force, ff, s0 = _case("random_walls_field_x4")
    ref = _gpu_run(shape, tau, s0, 5, flags=flags, uw=uw, force_field=ff, cells_per_lane=1)
    got = _gpu_run(shape, tau, s0, 5, flags=flags, uw=uw, force_field=ff, cells_per_lane=4, block=block)
    fl = flags == 0
    np.testing.assert_array_equal(got[:, fl], ref[:, fl])


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_16bit_one_step_matches_rounded_oracle(storage):
    shape, tau = (45, 21, 13), 0.7
    N = int(np.prod(shape))
    flags = W.random_flags(N, seed=31, solid_fraction=0.15, moving_fraction=0.03)
    h, plain = _offset_state(N, 32, storage)
    _, Wt, _ = oracle.tables()
    got = _gpu_run(shape, tau, plain, 1, flags=flags, uw=(0.04, 0.0, -0.02), force=(1e-5, 0, 2e-5),
                   storage=storage)
    olat = oracle_lattice(shape, tau, flags=flags, uw=(0.04, 0.0, -0.02), force=(1e-5, 0, 2e-5))
    ref = olat.step(Wt[:, None] + h)
    ref_q = oracle.quantize(ref, storage)
    fl = flags == 0
    hq = np.abs(ref_q - Wt[:, None])[:, fl]
    # one unit in the last place of the 16-bit format at each offset
    mant = 10 if storage == "f16" else 7
    emin = -14 if storage == "f16" else -126
    ulp = 2.0 ** (np.maximum(np.floor(np.log2(np.maximum(hq, 1e-300))), emin) - mant)
    diff = np.abs(got[:, fl].astype(np.float64) - ref_q[:, fl])
    # plus the FP32 representation of w_i + h (one FP32 ulp at w_0 = 1/3 is 3e-8)
    rep = 4e-8
    assert np.all(diff <= ulp * 1.01 + rep), float(np.max((diff - rep) / ulp))
    same = np.mean(diff <= rep)
    print(f"{storage}: {same * 100:.3f}% of fluid populations identical to the rounded oracle")
    assert same > 0.99


def test_resume_is_bit_exact():
    from paper_1309_1983_amd import Lattice
    shape, tau, flags, uw, force, ff, s0 = _case("random_walls_field")
    for pattern in ("ab", "aa"):
        full = _gpu_run(shape, tau, s0, 9, flags=flags, uw=uw, force_field=ff, pattern=pattern)
        lat = _lattice(shape, tau, flags=flags, uw=uw, force_field=ff, pattern=pattern)
        lat.set_populations(torch.from_numpy(s0))
        lat.step(5)
        saved = lat.populations().cpu()
        lat.close()
        lat2 = _lattice(shape, tau, flags=flags, uw=uw, force_field=ff, pattern=pattern)
        lat2.set_populations(saved)
        lat2.step(4)
        got = lat2.populations().cpu().numpy()
        lat2.close()
        fl = flags == 0
        np.testing.assert_array_equal(got[:, fl], full[:, fl], err_msg=pattern)


def test_nonfinite_detection_and_errors():
    from paper_1309_1983_amd import LBMError, Lattice
    shape = (20, 10, 6)
    N = int(np.prod(shape))
    lat = Lattice(*shape, 0.7, check_interval=2)
    lat.step(4)
    lat.check_finite()
    f = lat.populations()
    f[5, 123] = float("nan")
    lat.set_populations(f)
    with pytest.raises(LBMError, match="NONFINITE"):
        lat.check_finite()
    with pytest.raises(LBMError, match="NONFINITE"):
        lat.step(2)
    with pytest.raises(LBMError, match="INVALID"):
        lat.step(-1)
    with pytest.raises(LBMError, match="INVALID"):
        lat.set_wall_velocity(0.5, 0, 0)
    with pytest.raises(LBMError, match="INVALID"):
        lat.set_tau(0.5)
    with pytest.raises(LBMError, match="STATE"):
        lat.step_times()
    lat.close()
    # an unstable run is caught by the periodic check
    flags = W.cavity_flags(16, 16, 16)
    lat = Lattice(16, 16, 16, 0.5001, flags=flags, check_interval=50)
    lat.set_wall_velocity(0.29)
    with pytest.raises(LBMError, match="NONFINITE"):
        lat.step(20000)
    lat.close()


def test_step_times_log():
    from paper_1309_1983_amd import Lattice
    lat = Lattice(64, 64, 64, 0.7, timing=64)
    lat.step(10)
    t = lat.step_times()
    assert len(t) == 10 and np.all(t > 0)
    lat.step(100)
    t = lat.step_times()
    assert len(t) == 64 and np.all(t > 0)
    assert len(lat.step_times()) == 0
    lat.close()


def test_mass_conserved_f32_cavity():
    """Closed cavity with a tangential lid conserves mass exactly; FP32
    rounding keeps the drift at round-off (host FP64 sums)."""
    from paper_1309_1983_amd import Lattice
    shape = (96, 80, 64)
    flags = W.cavity_flags(*shape)
    lat = Lattice(*shape, 0.6, flags=flags)
    lat.set_wall_velocity(0.1)
    fl = torch.from_numpy(flags == 0).cuda()
    m0 = lat.populations()[:, fl].double().sum().item()
    lat.step(500)
    m1 = lat.populations()[:, fl].double().sum().item()
    lat.close()
    assert abs(m1 / m0 - 1) <= 1e-6
