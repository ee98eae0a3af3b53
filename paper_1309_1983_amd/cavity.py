"""Lid-driven cubic cavity with on-site velocity walls: the validation
workload of Mawson & Revell, Section 5.

Every face of the cube is a wall of on-site velocity nodes; the nodes of the
top face (y = L, edges and corners included) move with the lid along +x, all
others are at rest. The walls lie on node planes, so a cavity of side L
lattice spacings has L + 1 nodes per side; one layer of solid cells outside
closes the box (L + 3 points per side in all).

Eq. (8) ties the lid speed u, the relaxation time tau, the Reynolds number Re
and the side L: u = (tau - 1/2) Re / (3 L), i.e. Re = u L / nu with
nu = (tau - 1/2) / 3. `run` fixes u and L and takes tau from Re.

The result holds the two centreline profiles used to validate the solver
(Section 5): u_x along the vertical line through the cavity centre
(x = z = L/2) and u_y along the horizontal line (y = z = L/2), both scaled by
the lid speed, against the position scaled by L.
"""
from __future__ import annotations

import dataclasses
import sys
import time

import numpy as np
import torch

from .lattice import Lattice

WALL, ONSITE, ONSITE_MOVING = 1, 3, 4


def tau_for(Re: float, L: int, u_lid: float) -> float:
    """Relaxation time from Eq. (8): tau = 1/2 + 3 u L / Re."""
    return 0.5 + 3.0 * u_lid * L / Re


def cavity_flags(L: int) -> np.ndarray:
    """Flags of the cavity of side L (even): (L+3)^3 points, x fastest."""
    if L < 2 or L % 2:
        raise ValueError(f"cavity side must be even and >= 2 (got {L})")
    n = L + 3
    f = np.zeros((n, n, n), dtype=np.uint8)      # [z][y][x]
    f[1:-1, 1:-1, 1:-1] = ONSITE
    f[2:-2, 2:-2, 2:-2] = 0
    f[1:-1, -2, 1:-1] = ONSITE_MOVING
    f[0, :, :] = f[-1, :, :] = WALL
    f[:, 0, :] = f[:, -1, :] = WALL
    f[:, :, 0] = f[:, :, -1] = WALL
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
    glups: float               # lattice updates per second / 1e9 (all (L+3)^3 points)

    def as_dict(self):
        d = dataclasses.asdict(self)
        for k in ("y", "ux", "x", "uy"):
            d[k] = [round(float(v), 6) for v in d[k]]
        return d


def _profiles(lat: Lattice, L: int, u_lid: float):
    n = L + 3
    m = 1 + L // 2
    _, u = lat.macros()
    u = u.reshape(3, n, n, n)                      # [c][z][y][x]
    ux = (u[0, m, 1:L + 2, m] / u_lid).double().cpu().numpy()
    uy = (u[1, m, m, 1:L + 2] / u_lid).double().cpu().numpy()
    return ux, uy


def run(Re: float, L: int, u_lid: float = 0.1, storage: str = "f32", tol: float = 1e-5,
        check_every: int | None = None, max_steps: int | None = None, log=None) -> CavityResult:
    """Runs the cavity from rest until the scaled centreline profiles change
    by less than `tol` between two checks `check_every` steps apart (default
    2L), or until `max_steps` (default 80 L / u_lid, i.e. 80 lid transit
    times). `log`: file for one progress line per check."""
    tau = tau_for(Re, L, u_lid)
    n = L + 3
    check_every = check_every or max(2 * L, 100)
    max_steps = max_steps or int(80 * L / u_lid)
    lat = Lattice(n, n, n, tau, flags=cavity_flags(L), storage=storage)
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
                        seconds=secs, glups=n ** 3 * steps / secs / 1e9)


def resolution_differences(results):
    """Max differences of the scaled centreline profiles between successive
    resolutions (L, 2L, ...), compared at the coarse nodes, and the observed
    order log2(d_k / d_{k+1})."""
    rs = sorted(results, key=lambda r: r.L)
    diffs = []
    for a, b in zip(rs, rs[1:]):
        if b.L != 2 * a.L:
            raise ValueError("resolutions must double")
        d = max(np.max(np.abs(a.ux - b.ux[::2])), np.max(np.abs(a.uy - b.uy[::2])))
        diffs.append(float(d))
    orders = [float(np.log2(d0 / d1)) for d0, d1 in zip(diffs, diffs[1:]) if d1 > 0]
    return diffs, orders


def _finite_doubling_runs(res):
    """The longest chain of finite results, ending at the largest finite side,
    whose sides double from one to the next (ascending)."""
    good = [r for r in sorted(res, key=lambda r: r.L) if r.finite]
    chain = good[-1:]
    for r in reversed(good[:-1]):
        if chain[0].L == 2 * r.L:
            chain.insert(0, r)
        else:
            break
    return chain


def validation(Re_list=(100, 400, 1000), sides=None, u_lid=0.1, log=sys.stderr):
    """The paper's three Reynolds numbers at successively doubled sides."""
    sides = sides or {100: (32, 64, 128), 400: (64, 128, 256), 1000: (64, 128, 256)}
    out = {}
    for Re in Re_list:
        res = [run(Re, L, u_lid=u_lid, log=log) for L in sides[Re]]
        chain = _finite_doubling_runs(res)
        diffs, orders = resolution_differences(chain) if len(chain) > 1 else ([], [])
        out[Re] = {"runs": res, "differences": diffs, "orders": orders}
    return out
