"""Shared helpers of the GPU parity tests (imported by tests only)."""
import numpy as np

import oracle
import workloads as W

Q = 19


def f32(x):
    return np.float32(x)


def fluid_rel_err(got, ref, flags):
    """max over fluid cells and directions of |got - ref| / |ref|."""
    fl = np.ones(ref.shape[1], dtype=bool) if flags is None else (np.asarray(flags) == 0)
    return float(np.max(np.abs(got[:, fl] - ref[:, fl]) / np.abs(ref[:, fl])))


def near_rest_state(N, seed, drho=0.01, umax=0.02):
    """FP64 equilibrium of random (rho, u) from the oracle, rounded to FP32."""
    s = oracle.init_equilibrium(N, W.random_density(N, seed, drho), W.random_velocity(N, seed + 1, umax))
    return s.astype(np.float32)


def oracle_lattice(shape, tau, flags=None, uw=(0, 0, 0), force=None, force_field=None):
    """Oracle lattice with every parameter rounded to FP32 first (the GPU's inputs)."""
    uw = np.asarray(uw, dtype=np.float32).astype(np.float64)
    fo = None if force is None else np.asarray(force, dtype=np.float32).astype(np.float64)
    ff = None if force_field is None else np.asarray(force_field, dtype=np.float32).astype(np.float64)
    return oracle.Lattice(*shape, float(np.float32(tau)), flags=flags, uw=uw, force=fo, force_field=ff)


def neighbourhood(shape, c, r):
    """Flat indices of the (2r+1)^3 periodic box around cell c, box order
    (x fastest), so box cell (r, r, r) is c itself."""
    nx, ny, nz = shape
    x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
    d = np.arange(-r, r + 1)
    zz, yy, xx = np.meshgrid((z + d) % nz, (y + d) % ny, (x + d) % nx, indexing="ij")
    return ((zz * ny + yy) * nx + xx).reshape(-1)


def oracle_sampled(shape, tau, flags, uw, s0_of, cells, nsteps, force=None):
    """Oracle populations after nsteps at the given cells. Each cell is
    evolved inside its own (2*nsteps+1)^3 neighbourhood box: the value at the
    box centre after nsteps depends only on cells inside the box, so the
    box's periodic wrap never reaches it. s0_of(indices) -> [19, k] FP64."""
    r = nsteps
    out = np.empty((Q, len(cells)))
    b = 2 * r + 1
    centre = (r * b + r) * b + r
    for k, c in enumerate(cells):
        idx = neighbourhood(shape, int(c), r)
        fl = None if flags is None else np.asarray(flags)[idx]
        lat = oracle_lattice((b, b, b), tau, flags=fl, uw=uw, force=force)
        out[:, k] = lat.run(s0_of(idx), nsteps)[:, centre]
    return out
