"""Lid-driven cubic cavity with on-site velocity walls: the validation
workload of Mawson & Revell, Section 5.

Every face of the cube is a wall of on-site velocity nodes; the nodes of the
top face (y = L, edges and corners included) move with the lid along +x, all
others are at rest. The walls lie on node planes, so a cavity of side L
lattice spacings has L + 1 nodes per side; one layer of solid cells outside
closes the box (L + 3 points per side in all, plus solid padding along x up
to a multiple of 4 points so that the vector step kernel applies).

Eq. (8) ties the lid speed u, the relaxation time tau, the Reynolds number Re
and the side L: u = (tau - 1/2) Re / (3 L), i.e. Re = u L / nu with
nu = (tau - 1/2) / 3. `run` takes Re, L and either u or tau.

With the on-site walls read as here, the scheme loses stability near
tau = 0.55 at these resolutions (the lid corners go first), so high Reynolds
numbers need large L, as in the paper.

The result holds the two centreline profiles used to validate the solver
(Section 5): u_x along the vertical line through the cavity centre
(x = z = L/2) and u_y along the horizontal line (y = z = L/2), both scaled by
the lid speed, against the position scaled by L.
"""
from __future__ import annotations

import dataclasses
import math
import sys
import time

import numpy as np
import torch

from .lattice import Lattice

WALL, ONSITE, ONSITE_MOVING = 1, 3, 4


def tau_for(Re: float, L: int, u_lid: float) -> float:
    """Relaxation time from Eq. (8): tau = 1/2 + 3 u L / Re."""
    return 0.5 + 3.0 * u_lid * L / Re


def lid_speed_for(Re: float, L: int, tau: float) -> float:
    """Lid speed from Eq. (8): u = (tau - 1/2) Re / (3 L)."""
    return (tau - 0.5) * Re / (3.0 * L)


def box_shape(L: int):
    """(nx, ny, nz) of the cavity of side L."""
    n = L + 3
    return (n + 3) // 4 * 4, n, n


def cavity_flags(L: int) -> np.ndarray:
    """Flags of the cavity of side L (even), x fastest: on-site walls on the
    node planes 1 and L + 1 of every axis, solid outside."""
    if L < 2 or L % 2:
        raise ValueError(f"cavity side must be even and >= 2 (got {L})")
    nx, n, _ = box_shape(L)
    f = np.full((n, n, nx), WALL, dtype=np.uint8)      # [z][y][x]
    f[1:-1, 1:-1, 1:n - 1] = ONSITE
    f[2:-2, 2:-2, 2:n - 2] = 0
    f[1:-1, -2, 1:n - 1] = ONSITE_MOVING
    return f.reshape(-1)


@dataclasses.dataclass
class CavityResult:
    Re: float
    L: int
    tau: float
    u_lid: float
    steps: int
    converged: bool
    residual: float            # last max change of the scaled profiles between checks
    finite: bool
    y: np.ndarray              # positions / L of the vertical centreline
    ux: np.ndarray             # u_x / u_lid along it
    x: np.ndarray              # positions / L of the horizontal centreline
    uy: np.ndarray             # u_y / u_lid along it
    seconds: float
    glups: float               # lattice updates per second / 1e9 (all points of the box)

    def as_dict(self):
        d = dataclasses.asdict(self)
        for k in ("y", "ux", "x", "uy"):
            d[k] = [round(float(v), 6) for v in d[k]]
        return d


def _profiles(lat: Lattice, L: int, u_lid: float):
    nx, n, _ = box_shape(L)
    m = 1 + L // 2
    _, u = lat.macros()
    u = u.reshape(3, n, n, nx)                     # [c][z][y][x]
    ux = (u[0, m, 1:L + 2, m] / u_lid).double().cpu().numpy()
    uy = (u[1, m, m, 1:L + 2] / u_lid).double().cpu().numpy()
    return ux, uy


def run(Re: float, L: int, u_lid: float | None = None, tau: float | None = None,
        storage: str = "f32", tol: float = 1e-5, check_every: int | None = None,
        max_steps: int | None = None, log=None) -> CavityResult:
    """Runs the cavity from rest until the scaled centreline profiles change
    by less than `tol` between two checks `check_every` steps apart (default
    2L), or until `max_steps` (default 80 L / u_lid, i.e. 80 lid transit
    times). Give the lid speed or tau (Eq. (8) gives the other; default lid
    speed 0.1). `log`: file for one progress line per check."""
    if u_lid is not None and tau is not None:
        raise ValueError("give u_lid or tau, not both")
    if tau is None:
        u_lid = 0.1 if u_lid is None else u_lid
        tau = tau_for(Re, L, u_lid)
    else:
        u_lid = lid_speed_for(Re, L, tau)
    nx, n, _ = box_shape(L)
    check_every = check_every or max(2 * L, 100)
    max_steps = max_steps or int(80 * L / u_lid)
    lat = Lattice(nx, n, n, tau, flags=cavity_flags(L), storage=storage)
    try:
        lat.set_wall_velocity(u_lid, 0.0, 0.0)
        prev_x, prev_y = _profiles(lat, L, u_lid)
        steps, converged, residual, finite = 0, False, float("inf"), True
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while steps < max_steps:
            k = min(check_every, max_steps - steps)
            lat.step(k)
            steps += k
            ux, uy = _profiles(lat, L, u_lid)
            if not (np.all(np.isfinite(ux)) and np.all(np.isfinite(uy))):
                finite = False
                break
            residual = float(max(np.max(np.abs(ux - prev_x)), np.max(np.abs(uy - prev_y))))
            prev_x, prev_y = ux, uy
            if log is not None:
                print(f"cavity Re={Re:g} L={L} step {steps} residual {residual:.3e}", file=log, flush=True)
            if residual < tol:
                converged = True
                break
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
    finally:
        lat.close()
    pos = np.arange(L + 1) / L
    return CavityResult(Re=Re, L=L, tau=tau, u_lid=u_lid, steps=steps, converged=converged,
                        residual=residual, finite=finite, y=pos, ux=prev_x, x=pos, uy=prev_y,
                        seconds=secs, glups=nx * n * n * steps / secs / 1e9)


def common_nodes(La: int, Lb: int):
    """Indices into the profiles of sides La and Lb (nodes k / L, k = 0..L)
    of the positions both grids hold: every node of the coarser grid when one
    side is a multiple of the other."""
    g = math.gcd(La, Lb)
    m = np.arange(g + 1)
    return m * (La // g), m * (Lb // g)


def resolution_differences(results, norm="max"):
    """Differences of the scaled centreline profiles between successive
    resolutions (ascending L), compared at the positions both grids hold, in
    the max norm or the root-mean-square ("rms") over both profiles; and the
    observed orders log(d_k / d_{k+1}) / log(r), where the two comparisons
    refine the side by the same ratio r."""
    rs = sorted(results, key=lambda r: r.L)
    diffs, ratios = [], []
    for a, b in zip(rs, rs[1:]):
        if b.L <= a.L:
            raise ValueError("resolutions must differ")
        ia, ib = common_nodes(a.L, b.L)
        e = np.concatenate([a.ux[ia] - b.ux[ib], a.uy[ia] - b.uy[ib]])
        diffs.append(float(np.max(np.abs(e)) if norm == "max" else np.sqrt(np.mean(e * e))))
        ratios.append(b.L / a.L)
    orders = [float(np.log(d0 / d1) / np.log(r0))
              for d0, d1, r0, r1 in zip(diffs, diffs[1:], ratios, ratios[1:]) if d1 > 0 and r0 == r1]
    return diffs, orders


def _finite_runs(res):
    """The finite results, ascending in L."""
    return [r for r in sorted(res, key=lambda r: r.L) if r.finite]


# (Re, sides, fixed parameter): diffusive scaling (tau fixed, u ~ 1/L) where
# the lid speed stays at or below about 0.1, else a fixed lid speed. Re 1000
# pairs L = 256 with L = 384 (3:2, compared at every second node of 256):
# below 256 it needs tau < 0.55, where the scheme is unstable, and L = 512
# would take about 15 minutes.
VALIDATION_CASES = (
    (100, (32, 64, 128), {"tau": 0.6}),
    (400, (128, 256), {"tau": 0.6}),
    (1000, (256, 384), {"u_lid": 0.1}),
)


def validation(cases=VALIDATION_CASES, log=sys.stderr):
    """The paper's three Reynolds numbers, each at two or three sides where
    the cost allows."""
    out = {}
    for Re, sides, fixed in cases:
        res = [run(Re, L, log=log, **fixed) for L in sides]
        chain = _finite_runs(res)
        diffs, orders = resolution_differences(chain) if len(chain) > 1 else ([], [])
        rms, rms_orders = resolution_differences(chain, "rms") if len(chain) > 1 else ([], [])
        out[Re] = {"runs": res, "differences": diffs, "orders": orders, "rms_differences": rms,
                   "rms_orders": rms_orders, "fixed": fixed}
    return out
