"""Long-run drift of the benchmarked workload against the FP64 oracle.

The 256^3 lid-driven cavity (tau 0.6, lid 0.1 along +x, from rest) is run for
1000 steps on the GPU with FP32, FP16-offset and BF16-offset storage (two
arrays), and by the oracle in FP64 on the host; every 100 steps the velocity
and density of all fluid points are compared, and after the last step every
population of the FP32 run. The oracle takes about 4 minutes on 16 host cores,
too long for the test suite, so this is a script (not collected by pytest):

    python3 -u tests/long_cavity_drift.py
"""
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import numpy as np
import torch
import oracle
import workloads as W
from tests.gpu_common import oracle_lattice
from paper_1309_1983_amd import Lattice


def main(n=256, tau=0.6, lid=0.1, T=1000, E=100):
    flags = W.cavity_flags(n, n, n)
    fl = (flags == 0).reshape(-1)
    gpu = {}
    for st in ("f32", "f16", "bf16"):
        lat = Lattice(n, n, n, tau, flags=flags, storage=st)
        lat.set_wall_velocity(lid)
        lat.init_equilibrium()
        us = []
        for k in range(T // E):
            lat.step(E)
            rho, u = lat.macros()
            us.append((rho.cpu().numpy()[fl].astype(np.float64), u.cpu().numpy()[:, fl].astype(np.float64)))
        f = lat.populations().cpu().numpy() if st == "f32" else None
        lat.close()
        gpu[st] = (us, f)
        print(f"gpu {st} done", flush=True)
    torch.cuda.empty_cache()
    print(f"oracle threads {oracle.num_threads()}", flush=True)
    olat = oracle_lattice((n, n, n), tau, flags=flags, uw=(lid, 0, 0))
    s = oracle.init_equilibrium(n ** 3)
    t0 = time.time()
    for k in range(T // E):
        s = olat.run(s, E)
        rho_o, u_o = olat.macros(s)
        rho_o = rho_o.reshape(-1)[fl]; u_o = u_o.reshape(3, -1)[:, fl]
        umax = float(np.max(np.abs(u_o)))
        line = f"step {(k + 1) * E:5d} ({time.time() - t0:6.1f} s) max|u| {umax:.4e}"
        for st in ("f32", "f16", "bf16"):
            rg, ug = gpu[st][0][k]
            du = np.abs(ug - u_o)
            line += f" | {st}: max|du|/max|u| {du.max() / umax:.3e} rms {np.sqrt((du ** 2).mean()) / umax:.3e} max|drho| {np.abs(rg - rho_o).max():.3e}"
        print(line, flush=True)
    f = gpu["f32"][1]
    err = 0.0
    for i in range(19):
        r = s[i].reshape(-1)[fl]
        err = max(err, float(np.max(np.abs(f[i][fl].astype(np.float64) - r) / np.abs(r))))
    print(f"step {T}: FP32 AB max rel |df| over all fluid points and directions = {err:.3e}", flush=True)


if __name__ == "__main__":
    main()
