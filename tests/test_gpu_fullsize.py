"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (default work-group shape).

- 256^3 lid-driven cavity: full-domain parity after 100 steps from a random
  near-rest state (every point, every direction, <= 1e-5), and the FP16/BF16
  offset errors against the same oracle run bounded;
- 256^3 and 512^3 lid-driven cavities: 3 steps from a random near-rest
  state, sampled points checked against the oracle evolved in each point's
  7^3 neighbourhood (exact: 3 pull steps only reach 3 points away);
- 512^3: 100 steps against the oracle on three 17^3 blocks (a lid corner,
  a lid edge, the centre) for FP32 two-array (<= 1e-5) and FP16-offset
  in-place storage; the in-place AA pattern equals the two-array pattern bit for bit
  (FP32), mass is conserved over 500 steps, and the FP16-offset AA run over
  500 steps is reported against the FP32 run (labelled as such);
- 128 x 128 x 256 sphere duct with body force: full-domain FP32 parity after
  100 steps (<= 1e-5), and the FP16/BF16 offset error against the oracle;
  after 2000 steps (the workload's length) the error of all three storages
  against the oracle is bounded at the accuracy stated for each.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import fluid_rel_err, near_rest_state, oracle_lattice, oracle_sampled

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1309_1983_amd
    paper_1309_1983_amd.lib()


def _sample_cells(n, flags, k, seed):
    rng = np.random.default_rng(seed)
    pts = [(1, 1, 1), (n - 2, n - 2, n - 2), (1, n - 2, 1), (n - 2, n - 2, 1), (2, n - 2, n // 2),
           (n // 2, n - 2, n // 2), (n // 2, n // 2, n // 2), (3, 5, 7), (4, 6, 8), (n - 5, 9, 11)]
    cells = [(z * n + y) * n + x for x, y, z in pts]
    cells += list(rng.integers(0, n ** 3, k))
    return np.array([c for c in cells if flags[c] == 0], dtype=np.int64)


@pytest.mark.timeout(600)
def test_cavity256_full_domain_100_steps():
    """The benchmarked workload (256^3 cavity, tau 0.6, lid 0.1 along +x, two
    arrays, default launch) against the FP64 oracle on every point after 100
    steps: FP32 within 1e-5, and the FP16/BF16-offset runs within the
    accuracy stated for them (measured on MI355X: 3.0e-4 and 2.5e-3 relative
    in f; bounds about three times that). The start is a random near-rest
    equilibrium rather than rest, so that every point carries a non-trivial
    state from the first step."""
    from paper_1309_1983_amd import Lattice
    n, tau, lid, steps = 256, 0.6, 0.1, 100
    flags = W.cavity_flags(n, n, n)
    N = n ** 3
    s0 = near_rest_state(N, 31, 0.01, 0.02)
    got = {}
    for storage in ("f32", "f16", "bf16"):
        lat = Lattice(n, n, n, tau, flags=flags, storage=storage)
        lat.set_wall_velocity(lid)
        lat.set_populations(torch.from_numpy(s0))
        lat.step(steps)
        got[storage] = lat.populations().cpu().numpy()
        lat.close()
    torch.cuda.empty_cache()
    olat = oracle_lattice((n, n, n), tau, flags=flags, uw=(lid, 0, 0))
    ref = olat.run(s0.astype(np.float64), steps)
    del s0
    fl = flags == 0
    err = {k: 0.0 for k in got}
    for i in range(19):    # one direction at a time keeps the host copies small
        r = ref[i, fl]
        for k, f in got.items():
            err[k] = max(err[k], float(np.max(np.abs(f[i, fl].astype(np.float64) - r) / np.abs(r))))
    print(f"256^3 cavity, all {int(fl.sum())} fluid points after {steps} steps: max rel |df| = "
          f"{err['f32']:.3e} (FP32), {err['f16']:.3e} (FP16 offsets), {err['bf16']:.3e} (BF16 offsets)")
    assert err["f32"] <= 1e-5
    assert err["f16"] <= 1e-3
    assert err["bf16"] <= 1e-2


@pytest.mark.parametrize("n,tau,lid", [(256, 0.6, 0.1), (512, 0.55, 0.05)])
def test_cavity_full_size_sampled(n, tau, lid):
    from paper_1309_1983_amd import Lattice
    N = n ** 3
    flags = W.cavity_flags(n, n, n)
    rho = W.random_density(N, 1, 0.01).astype(np.float32)
    u = W.random_velocity(N, 2, 0.02).astype(np.float32)
    steps = 3
    lat = Lattice(n, n, n, tau, flags=flags)
    lat.set_wall_velocity(lid)
    lat.init_equilibrium(torch.from_numpy(rho), torch.from_numpy(u))
    lat.step(steps)
    cells = _sample_cells(n, flags, 300, 3)
    got = lat.populations()[:, torch.from_numpy(cells).cuda()].cpu().numpy().astype(np.float64)
    lat.close()
    torch.cuda.empty_cache()
    rho64, u64 = rho.astype(np.float64), u.astype(np.float64)

    def s0_of(idx):
        return oracle.init_equilibrium(len(idx), rho64[idx], u64[:, idx]).astype(np.float32).astype(np.float64)

    ref = oracle_sampled((n, n, n), tau, flags, (lid, 0, 0), s0_of, cells, steps)
    err = float(np.max(np.abs(got - ref) / np.abs(ref)))
    print(f"{n}^3 cavity, {len(cells)} sampled points after {steps} steps: max rel |df| = {err:.3e}")
    assert err <= 1e-5


@pytest.mark.timeout(900)
def test_cavity512_100_steps_sampled_vs_oracle():
    """512^3 cavity (tau 0.55, lid 0.05), 100 steps from a random near-rest
    equilibrium, in the benchmarked launch: the FP32 two-array state against
    the FP64 oracle at every point of three 17^3 blocks, centred on a lid
    corner, the middle of a lid edge and the cavity centre (<= 1e-5). The
    oracle evolves each block inside a 217^3 neighbourhood taken from the
    GPU's own initial state: 100 pull steps reach 100 points, so the block
    (8 points around the centre) never sees the neighbourhood's wrap. The
    FP16-offset in-place run from the same (rho, u) is compared with the same
    oracle values and bounded by its format's resolution."""
    from paper_1309_1983_amd import Lattice
    from tests.gpu_common import neighbourhood
    n, tau, lid, steps, r = 512, 0.55, 0.05, 100, 8
    N = n ** 3
    flags = W.cavity_flags(n, n, n)
    centres = [(r + 1, n - 2 - r, r + 1), (n // 2, n - 2 - r, r + 1), (n // 2, n // 2, n // 2)]
    rho = torch.from_numpy(W.random_density(N, 1, 0.01).astype(np.float32))
    u = torch.from_numpy(W.random_velocity(N, 2, 0.02).astype(np.float32))
    lat = Lattice(n, n, n, tau, flags=flags)
    lat.set_wall_velocity(lid)
    lat.init_equilibrium(rho, u)
    f0 = lat.populations()
    R = steps + r
    b = 2 * R + 1
    d = np.arange(-r, r + 1)
    zz, yy, xx = np.meshgrid(R + d, R + d, R + d, indexing="ij")
    inner = ((zz * b + yy) * b + xx).reshape(-1)        # the 17^3 block in box order
    cells, refs = [], []
    for x, y, z in centres:
        c = (z * n + y) * n + x
        idx = neighbourhood((n, n, n), c, R)
        box0 = f0[:, torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
        olat = oracle_lattice((b, b, b), tau, flags=flags[idx], uw=(lid, 0, 0))
        out = olat.run(box0, steps)[:, inner]
        keep = flags[idx[inner]] == 0
        cells.append(idx[inner][keep])
        refs.append(out[:, keep])
        print(f"oracle block at ({x}, {y}, {z}) done", flush=True)
    del f0
    torch.cuda.empty_cache()
    cells = np.concatenate(cells)
    ref = np.concatenate(refs, axis=1)
    lat.step(steps)
    ci = torch.from_numpy(cells).cuda()
    got = lat.populations()[:, ci].cpu().numpy().astype(np.float64)
    lat.close()
    torch.cuda.empty_cache()
    err = float(np.max(np.abs(got - ref) / np.abs(ref)))
    h = Lattice(n, n, n, tau, flags=flags, storage="f16", pattern="aa")
    h.set_wall_velocity(lid)
    h.init_equilibrium(rho, u)
    h.step(steps)
    g16 = h.populations()[:, ci].cpu().numpy().astype(np.float64)
    h.close()
    torch.cuda.empty_cache()
    err16 = float(np.max(np.abs(g16 - ref) / np.abs(ref)))
    print(f"512^3 cavity, {len(cells)} points after {steps} steps: FP32 AB max rel |df| = {err:.3e}; "
          f"FP16-offset AA max rel |df| = {err16:.3e}")
    assert len(cells) > 3 * 4000
    assert err <= 1e-5
    assert err16 <= 2e-3


def test_cavity512_aa_equals_ab_and_f16_report():
    from paper_1309_1983_amd import Lattice
    n, tau, lid = 512, 0.55, 0.05
    flags = W.cavity_flags(n, n, n)
    fl = torch.from_numpy(flags == 0).cuda()
    ab = Lattice(n, n, n, tau, flags=flags)
    ab.set_wall_velocity(lid)
    aa = Lattice(n, n, n, tau, flags=flags, pattern="aa")
    aa.set_wall_velocity(lid)
    ab.step(5)
    aa.step(5)   # odd count: AA state in its shifted layout
    fa, fb = ab.populations(), aa.populations()
    assert torch.equal(fa[:, fl], fb[:, fl])
    del fb
    aa.close()
    m0 = float(fa[:, fl].double().sum())
    del fa
    torch.cuda.empty_cache()
    ab.step(495)
    f32 = ab.populations()
    m1 = float(f32[:, fl].double().sum())
    assert abs(m1 / m0 - 1) < 1e-6
    _, u32 = ab.macros()
    ab.close()
    del f32
    torch.cuda.empty_cache()
    h = Lattice(n, n, n, tau, flags=flags, storage="f16", pattern="aa")
    h.set_wall_velocity(lid)
    h.step(500)
    _, u16 = h.macros()
    h.close()
    du = (u16 - u32)[:, fl]
    umax = float(u32[:, fl].abs().max())
    rms = float(du.pow(2).mean().sqrt()) / umax
    mx = float(du.abs().max()) / umax
    print(f"512^3 cavity, 500 steps: FP16-offset AA vs FP32 AB: max |du|/max|u| = {mx:.3e}, "
          f"RMS = {rms:.3e}; FP32 mass drift {m1 / m0 - 1:.2e}")
    assert mx < 0.05


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_sphere_duct_full_size_vs_oracle(storage):
    from paper_1309_1983_amd import Lattice
    nx, ny, nz, tau = 128, 128, 256, 0.7
    flags = W.sphere_duct_flags(nx, ny, nz, seed=20130909, solid_fraction=0.10)
    N = flags.size
    force = (0.0, 0.0, 1e-6)
    s0 = near_rest_state(N, 17, 0.005, 0.01)
    steps = 100
    lat = Lattice(nx, ny, nz, tau, flags=flags, storage=storage)
    lat.set_force(force)
    lat.set_populations(torch.from_numpy(s0))
    lat.step(steps)
    got = lat.populations().cpu().numpy().astype(np.float64)
    _, ug = lat.macros()
    lat.close()
    olat = oracle_lattice((nx, ny, nz), tau, flags=flags, force=force)
    ref = olat.run(s0.astype(np.float64), steps)
    _, uo = olat.macros(ref)
    err = fluid_rel_err(got, ref, flags)
    fl = flags == 0
    du = ug.cpu().numpy()[:, fl] - uo[:, fl]
    umax = np.abs(uo[:, fl]).max()
    print(f"spheres 128x128x256 {storage}: max rel |df| {err:.3e}, max |du|/max|u| "
          f"{np.abs(du).max() / umax:.3e}, RMS {np.sqrt((du ** 2).mean()) / umax:.3e}")
    if storage == "f32":
        assert err <= 1e-5
    else:
        # 16-bit offsets: reported; bounded by a few units of the format's
        # resolution relative to the offsets' size
        assert err <= (2e-3 if storage == "f16" else 2e-2)


@pytest.mark.timeout(900)
def test_sphere_duct_2000_steps_error_report():
    """The sphere-duct workload over its full 2000 steps from rest: velocity
    and population error of FP32, FP16-offset and BF16-offset storage
    against the FP64 oracle (reported; FP32 bounded)."""
    from paper_1309_1983_amd import Lattice
    nx, ny, nz, tau, steps = 128, 128, 256, 0.7, 2000
    flags = W.sphere_duct_flags(nx, ny, nz, seed=20130909, solid_fraction=0.10)
    N = flags.size
    fl = flags == 0
    force = (0.0, 0.0, 1e-6)
    olat = oracle_lattice((nx, ny, nz), tau, flags=flags, force=force)
    ref = olat.run(oracle.init_equilibrium(N), steps)
    _, uo = olat.macros(ref)
    umax = np.abs(uo[:, fl]).max()
    errs = {}
    for storage in ("f32", "f16", "bf16"):
        lat = Lattice(nx, ny, nz, tau, flags=flags, storage=storage)
        lat.set_force(force)
        lat.step(steps)
        got = lat.populations().cpu().numpy().astype(np.float64)
        _, ug = lat.macros()
        lat.close()
        du = ug.cpu().numpy()[:, fl] - uo[:, fl]
        errs[storage] = (fluid_rel_err(got, ref, flags), np.abs(du).max() / umax,
                         np.sqrt((du ** 2).mean()) / umax)
        print(f"spheres {storage}, {steps} steps from rest: max rel |df| {errs[storage][0]:.3e}, "
              f"max |du|/max|u| {errs[storage][1]:.3e}, RMS {errs[storage][2]:.3e} (max|u| {umax:.3e})")
    assert errs["f32"][0] <= 1e-5 and errs["f32"][1] <= 1e-3
    # 16-bit offsets: the accuracy stated for this workload (MI355X: FP16
    # 2.1e-3 max / 3.5e-4 RMS, BF16 3.5e-2 max / 7.3e-3 RMS of max|u|), with
    # some headroom
    assert errs["f16"][1] <= 5e-3 and errs["f16"][2] <= 1e-3
    assert errs["bf16"][1] <= 7e-2 and errs["bf16"][2] <= 1.5e-2
