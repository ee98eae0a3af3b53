"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds geometry (solid flags), initial macroscopic fields, force
fields and random population arrays. It contains none of the lattice
Boltzmann arithmetic: no velocity set, no weights, no equilibrium. Both the
HIP path and the oracle receive exactly these arrays.

Flag values: 0 = fluid, 1 = resting wall, 2 = moving wall, 3 = on-site
velocity node at rest, 4 = on-site velocity node moving with the wall
velocity (walls 1 and 2 are solid cells; on-site nodes are fluid nodes that
lie on the wall). Arrays are flat in
the order x fastest, then y, then z (idx = (z*ny + y)*nx + x); vector fields
are [3][N] (component slowest).
"""
from __future__ import annotations

import numpy as np

FLUID, WALL, MOVING_WALL, ONSITE, ONSITE_MOVING = 0, 1, 2, 3, 4


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def cavity_flags(nx, ny, nz):
    """Lid-driven cavity: a one-cell wall frame on every face of the box; the
    whole y = ny-1 face (edges included) is the moving lid."""
    f = np.zeros((nz, ny, nx), dtype=np.uint8)
    f[0, :, :] = WALL
    f[-1, :, :] = WALL
    f[:, 0, :] = WALL
    f[:, :, 0] = WALL
    f[:, :, -1] = WALL
    f[:, -1, :] = MOVING_WALL
    return f.reshape(-1)


def duct_flags(nx, ny, nz):
    """Square duct along z: walls on the x = 0, nx-1 and y = 0, ny-1 faces,
    periodic in z."""
    f = np.zeros((nz, ny, nx), dtype=np.uint8)
    f[:, 0, :] = WALL
    f[:, -1, :] = WALL
    f[:, :, 0] = WALL
    f[:, :, -1] = WALL
    return f.reshape(-1)


def channel_flags(n_fluid, nx=1, nz=1, lid=False):
    """Plane channel between walls at y = 0 and y = n_fluid + 1 (fluid rows
    y = 1..n_fluid), periodic in x and z. lid=True makes the top wall move."""
    ny = n_fluid + 2
    f = np.zeros((nz, ny, nx), dtype=np.uint8)
    f[:, 0, :] = WALL
    f[:, -1, :] = MOVING_WALL if lid else WALL
    return f.reshape(-1)


def onsite_cavity_flags(nx, ny, nz):
    """Lid-driven cavity with on-site velocity nodes: a one-cell solid frame on
    every face of the box, and the next layer inward made of on-site nodes.
    The on-site nodes of the y = ny-2 plane (its edges and corners included)
    move with the lid; all other on-site nodes are at rest. The walls lie on
    the node planes x = 1, nx-2 (and likewise in y, z), so the cavity side is
    nx - 3 lattice spacings."""
    f = np.zeros((nz, ny, nx), dtype=np.uint8)
    f[1:-1, 1:-1, 1:-1] = ONSITE
    f[2:-2, 2:-2, 2:-2] = FLUID
    f[1:-1, -2, 1:-1] = ONSITE_MOVING
    f[0, :, :] = WALL
    f[-1, :, :] = WALL
    f[:, 0, :] = WALL
    f[:, -1, :] = WALL
    f[:, :, 0] = WALL
    f[:, :, -1] = WALL
    return f.reshape(-1)


def onsite_channel_flags(h, nx=1, nz=1, lid=False):
    """Plane channel whose walls are on-site nodes at y = 1 and y = h + 1
    (wall distance h), with solid cells at y = 0 and y = h + 2, periodic in x
    and z. lid=True makes the top nodes move with the wall velocity."""
    ny = h + 3
    f = np.zeros((nz, ny, nx), dtype=np.uint8)
    f[:, 0, :] = WALL
    f[:, 1, :] = ONSITE
    f[:, -2, :] = ONSITE_MOVING if lid else ONSITE
    f[:, -1, :] = WALL
    return f.reshape(-1)


def sphere_duct_flags(nx, ny, nz, seed, solid_fraction=0.10, rmin=4.0, rmax=8.0):
    """Duct with random spherical obstacles.

    Centres are uniform in the duct interior, radii uniform in [rmin, rmax]
    (numpy PCG64 from `seed`); a cell is solid when its squared distance to a
    centre is <= r^2, using the minimum image along the periodic z axis.
    Spheres are added until solids cover >= solid_fraction of the interior.
    """
    rng = np.random.default_rng(seed)
    f = duct_flags(nx, ny, nz).reshape(nz, ny, nx)
    interior = (nx - 2) * (ny - 2) * nz
    solid = np.zeros((nz, ny, nx), dtype=bool)
    count = 0
    while count < solid_fraction * interior:
        cx = rng.uniform(1, nx - 2)
        cy = rng.uniform(1, ny - 2)
        cz = rng.uniform(0, nz)
        r = rng.uniform(rmin, rmax)
        x0, x1 = max(1, int(np.floor(cx - r))), min(nx - 2, int(np.ceil(cx + r)))
        y0, y1 = max(1, int(np.floor(cy - r))), min(ny - 2, int(np.ceil(cy + r)))
        zs = np.arange(int(np.floor(cz - r)), int(np.ceil(cz + r)) + 1)
        xs = np.arange(x0, x1 + 1)
        ys = np.arange(y0, y1 + 1)
        dz = zs - cz
        zw = np.mod(zs, nz)
        Z, Y, X = np.meshgrid(dz, ys - cy, xs - cx, indexing="ij")
        inside = X * X + Y * Y + Z * Z <= r * r
        for k, zz in enumerate(zw):
            solid[zz, y0:y1 + 1, x0:x1 + 1] |= inside[k]
        count = int(solid[:, 1:ny - 1, 1:nx - 1].sum())
    f[solid & (f == FLUID)] = WALL
    return f.reshape(-1)


def taylor_green_velocity(nx, ny, nz, u0, L=None):
    """u = u0 (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0), k = 2 pi / L,
    at integer cell coordinates. Returns [3][N] float64."""
    L = nx if L is None else L
    k = 2.0 * np.pi / L
    x, y, z = _grid(nx, ny, nz)
    ux = u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    uy = -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    return np.stack([ux, uy, np.zeros_like(ux)])


def shear_wave_velocity(nx, ny, nz, u0, axis_u=0, axis_k=1):
    """u_{axis_u} = u0 sin(2 pi c / n) along coordinate axis_k. [3][N] float64."""
    coords = _grid(nx, ny, nz)
    n = (nx, ny, nz)[axis_k]
    u = np.zeros((3, nx * ny * nz))
    u[axis_u] = u0 * np.sin(2.0 * np.pi * coords[axis_k] / n)
    return u


def random_velocity(N, seed, umax):
    rng = np.random.default_rng(seed)
    return rng.uniform(-umax, umax, size=(3, N))


def random_density(N, seed, amp):
    rng = np.random.default_rng(seed)
    return 1.0 + rng.uniform(-amp, amp, size=N)


def random_force_field(N, seed, fmax):
    """Each component i.i.d. U(-1, 1) * fmax / sqrt(3), so |F| <= fmax."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(3, N)) * (fmax / np.sqrt(3.0))


def random_values(shape, seed, lo=0.0, hi=1.0, dtype=np.float32):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape).astype(dtype)


def random_flags(N, seed, solid_fraction, moving_fraction=0.0):
    rng = np.random.default_rng(seed)
    r = rng.uniform(size=N)
    f = np.zeros(N, dtype=np.uint8)
    f[r < solid_fraction] = WALL
    f[r < moving_fraction] = MOVING_WALL
    return f


# The five workloads, with the physical parameters they are quoted on.
CONFIGS = {
    "tgv32": dict(shape=(32, 32, 32), tau=0.8, u0=0.05, steps=100, storage="f32"),
    "cavity256": dict(shape=(256, 256, 256), tau=0.6, lid=0.1, steps=1000, storage="f32"),
    "spheres128x128x256": dict(shape=(128, 128, 256), tau=0.7, force=1e-6, steps=2000,
                               seed=20130909, solid_fraction=0.10),
    "adjoint64": dict(shape=(64, 64, 64), tau=0.7, T=200, K=20, fmax=1e-5, seed_force=1,
                      seed_target=2),
    "cavity512": dict(shape=(512, 512, 512), tau=0.55, lid=0.05, steps=500),
}
