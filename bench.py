#!/usr/bin/env python3
"""Throughput benchmark of the D3Q19 step on one MI355X.

Workload (default): D3Q19 BGK lid-driven cavity 256^3, FP32 populations in two
arrays, tau 0.6, lid velocity 0.1 in x, from rest. A step is one fused pull
stream-collide pass over all 256^3 points (Mawson & Revell, Algorithm 3).
MLUPS counts every lattice point, solid or fluid (the paper's convention).

Printed JSON line (rank 0, stdout): the contract fields, plus
  roofline      achieved HBM GB/s of the step kernel from the algorithmic
                152 B per point (19 loads + 19 stores of 4 B, Section 4.1)
                over its average duration, vs the 8 TB/s MI355X peak;
  cpu_baseline  the FP64 oracle timed on the host cores on a bounded sample;
  extra         16-bit offset storage (two-array and in-place AA) rates, the
                adjoint reverse sweep rates (256^3 and 64^3), the measured
                copy ceiling, the access pattern's own ceilings (the step
                without collision; its 19-plane streams without shifts), the
                other workload configurations, and the per-step time
                distribution with its periodogram peak.
Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, decimal GB/s
BYTES_PER_POINT = {"f32": 152, "f16": 76, "bf16": 76}   # 19 loads + 19 stores
MACROS_BYTES = 16   # rho and u stored every step (Section 4.1: 152 -> 168 B)
FORCE_FIELD_BYTES = 12   # a per-point force [3][N] FP32 read by every step
# reverse step: reads b 76, s 76 and F 12; writes b 76; grad_F read and written 24
ADJOINT_REVERSE_BYTES = 264
# per point and time step of the reverse sweep: the recompute step with the
# force field (152 + 12) plus the reverse step
ADJOINT_BYTES_PER_POINT = BYTES_PER_POINT["f32"] + FORCE_FIELD_BYTES + ADJOINT_REVERSE_BYTES


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _code_of(text):
    """Source text without // comments, trailing blanks and blank lines: what
    the compiler sees of the step kernels (the hashed files use no block
    comments and no // inside string literals)."""
    lines = (line.split("//", 1)[0].rstrip() for line in text.splitlines())
    return "\n".join(line for line in lines if line)


def kernel_source_hash():
    """Hash of the step kernels' code (comments and layout left out), stored
    with the counter summaries so that the benchmark reports traffic only for
    the kernels the counters were taken on."""
    h = hashlib.sha256()
    for name in ("d3q19.hpp", "kernels_step.hip", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_1309_1983_amd", "csrc", name), encoding="utf-8") as fh:
            h.update(_code_of(fh.read()).encode())
    return h.hexdigest()[:16]


def _kernel_key(name):
    """Kernel name without its parameter list (the template arguments stay)."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    if not name.endswith(")"):
        return name
    depth = 0
    for k in range(len(name) - 1, -1, -1):   # the last parenthesised group
        if name[k] == ")":
            depth += 1
        elif name[k] == "(":
            depth -= 1
            if depth == 0:
                return name[:k]
    return name


def load_traffic(workload, kernel_name):
    """HBM bytes per launch of `kernel_name` from the committed rocprofv3
    counter summary of `workload`, if it was taken on the current kernel
    source (else None)."""
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    for k in d.get("kernels", []):
        if k["kernel"] == _kernel_key(kernel_name):
            return k["hbm_bytes_per_launch"]
    return None


# ---- rocprofv3 counter summaries (run on the host after the counter passes) ----
# Every pass is `rocprofv3 --pmc <counters> --output-format csv -d <DIR>/<pass>_<what>
# -o run -- python3 bench.py --profile <what> --steps 10`, one pass per counter set:
PMC_PASSES = {
    "fetch": ["FETCH_SIZE"],
    "write": ["WRITE_SIZE"],
    "rdreq": ["TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_sum"],
    "wrreq": ["TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum"],
    "hit": ["TCC_HIT_sum", "TCC_MISS_sum"],
}
PMC_WORKLOADS = {   # --profile workload -> (summary name, lattice points)
    "cavity": ("cavity256", 256 ** 3),
    "spheres": ("spheres128x128x256", 128 * 128 * 256),
    "adjoint": ("adjoint256", 256 ** 3),
}
COPY_BYTES_EACH_WAY = 2 << 30   # the copy probes of --profile copy: 2 GiB read, 2 GiB written


def _pmc_table(path):
    """{kernel key: {counter: [per-dispatch values]}} from one pass's CSV."""
    import csv
    out = {}
    with open(os.path.join(path, "run_counter_collection.csv")) as fh:
        for r in csv.DictReader(fh):
            k = _kernel_key(r["Kernel_Name"])
            if k.startswith("at::") or "rocclr" in k or "__amd_" in k:
                continue
            out.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return out


def _algorithmic_bytes_per_point(kernel):
    """State bytes one launch must move per lattice point (Section 4.1): 19
    loads and 19 stores of the storage width for a step, plus the force field
    when the step reads one; 264 B for the reverse step; None otherwise."""
    if kernel.startswith("lbmk::k_adj_stepv"):
        return ADJOINT_REVERSE_BYTES
    for pre in ("lbmk::k_step_abv<", "lbmk::k_step_aa0<", "lbmk::k_step_aa1<"):
        if kernel.startswith(pre):
            args = [a.strip() for a in kernel[len(pre):-1].split(",")]
            width = 4 if args[0].endswith("StF32") else 2
            field = args[1] == "2"
            return 2 * 19 * width + (FORCE_FIELD_BYTES if field else 0)
    return None


def pmc_summary(root, out_dir):
    """Write profiles/pmc_traffic_<workload>.json from the counter passes under
    `root`: per kernel the FETCH_SIZE / WRITE_SIZE figures scaled by what the
    same counters read for the copy probes of known size, the exact EA
    request bytes (128/64/32-byte read requests, 64/32-byte write requests)
    and the L2 hit rate, all per dispatch."""
    def mean(v):
        return sum(v) / len(v)

    rel = os.path.relpath(root, ROOT) if os.path.abspath(root).startswith(ROOT + os.sep) else root
    cal = {p: _pmc_table(os.path.join(root, f"{p}_copy")) for p in ("fetch", "write")}
    copies = sorted(cal["fetch"])
    fetch_kib = mean([mean(cal["fetch"][k]["FETCH_SIZE"]) for k in copies])
    write_kib = mean([mean(cal["write"][k]["WRITE_SIZE"]) for k in copies])
    f_fac = COPY_BYTES_EACH_WAY / (fetch_kib * 1024)
    w_fac = COPY_BYTES_EACH_WAY / (write_kib * 1024)
    calibration = {"copy_kernels": copies, "copy_bytes_each_way": COPY_BYTES_EACH_WAY,
                   "copy_fetch_size_kib_per_dispatch": round(fetch_kib, 1),
                   "copy_write_size_kib_per_dispatch": round(write_kib, 1),
                   "fetch_factor": round(f_fac, 5), "write_factor": round(w_fac, 5)}
    written = []
    for what, (name, npts) in PMC_WORKLOADS.items():
        t = {p: _pmc_table(os.path.join(root, f"{p}_{what}")) for p in PMC_PASSES}
        kernels = []
        for k in t["fetch"]:
            c = {}
            for p in PMC_PASSES:
                for cn, v in t[p].get(k, {}).items():
                    c[cn] = mean(v)
            rd = f_fac * c["FETCH_SIZE"] * 1024
            wr = w_fac * c.get("WRITE_SIZE", 0.0) * 1024
            e = {"kernel": k, "dispatches": len(t["fetch"][k]["FETCH_SIZE"]),
                 "fetch_size_kib": round(c["FETCH_SIZE"], 1), "write_size_kib": round(c.get("WRITE_SIZE", 0.0), 1),
                 "hbm_read_bytes": round(rd), "hbm_write_bytes": round(wr), "hbm_bytes_per_launch": round(rd + wr)}
            if "TCC_EA0_RDREQ_sum" in c:
                e["ea_read_bytes_from_request_sizes"] = round(
                    32 * c["TCC_EA0_RDREQ_32B_sum"] + 64 * c["TCC_EA0_RDREQ_64B_sum"]
                    + 128 * c["TCC_EA0_RDREQ_128B_sum"])
            if "TCC_EA0_WRREQ_sum" in c:
                e["ea_write_bytes_from_request_sizes"] = round(
                    64 * c["TCC_EA0_WRREQ_64B_sum"] + 32 * (c["TCC_EA0_WRREQ_sum"] - c["TCC_EA0_WRREQ_64B_sum"]))
            if "TCC_HIT_sum" in c:
                e["l2_hit_rate"] = round(c["TCC_HIT_sum"] / max(1.0, c["TCC_HIT_sum"] + c["TCC_MISS_sum"]), 4)
            bpp = _algorithmic_bytes_per_point(k)
            if bpp is not None:
                e["algorithmic_bytes_per_launch"] = bpp * npts
                e["traffic_over_algorithmic"] = round((rd + wr) / (bpp * npts), 4)
            kernels.append(e)
        doc = {"workload": name, "kernel_source_hash": kernel_source_hash(),
               "commands": [f"rocprofv3 --pmc {' '.join(cs)} --output-format csv -d {rel}/{p}_{w} "
                            f"-o run -- python3 bench.py --profile {w} --steps 10"
                            for w in (what, "copy") for p, cs in PMC_PASSES.items()
                            if w == what or p in ("fetch", "write")]
                           + [f"python3 bench.py --pmc-summary {rel}"],
               "calibration": calibration, "kernels": kernels}
        path = os.path.join(out_dir, f"pmc_traffic_{name}.json")
        with open(path, "w") as fh:
            json.dump(doc, fh, indent=1)
            fh.write("\n")
        written.append(path)
    return written


def time_steps(lat, steps, torch, stream_only=False):
    """Average ms per step over `steps` back-to-back launches, with HIP events
    recorded on the lattice's stream (the stream the kernels run on).
    stream_only: the streaming half alone (no collision)."""
    s = lat.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    if stream_only:
        lat.stream_only(steps)
    else:
        lat.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cavity_lattice(n, storage, pattern, tau, lid, block=None, cells_per_lane=0, onsite=False):
    import workloads as W
    from paper_1309_1983_amd import Lattice
    flags = W.onsite_cavity_flags(n, n, n) if onsite else W.cavity_flags(n, n, n)
    lat = Lattice(n, n, n, tau, flags=flags, storage=storage, pattern=pattern, block=block,
                  cells_per_lane=cells_per_lane)
    lat.set_wall_velocity(lid)
    return lat


def copy_ceiling(torch, gib=2.0, reps=20):
    from paper_1309_1983_amd import copy_f32
    n = int(gib * (1 << 30) / 4)
    a = torch.empty(n, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a)
    for _ in range(3):
        copy_f32(a, b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        copy_f32(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    assert torch.equal(a[:1000], b[:1000])
    del a, b
    torch.cuda.empty_cache()
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def pattern_ceilings(torch, n, reps=20):
    """Bandwidth of the step's own memory streams without its stencil: the 19
    planes of each z-slab copied, read and written in the step's layout and
    launch shape (lbm_study_planes), all accesses aligned."""
    from paper_1309_1983_amd import study
    N = n ** 3
    a = torch.rand(19 * N, device="cuda")
    b = torch.empty_like(a)
    sink = torch.zeros(4, device="cuda")
    out = {}
    for mode, nbytes in (("copy", 2 * 19 * N * 4), ("read", 19 * N * 4), ("write", 19 * N * 4)):
        ms = _time_ms(torch, lambda: study.planes(mode, a, b, sink, n, n, n), reps)
        out[f"planes19_{mode}_gbs"] = round(nbytes / (ms * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def step_time_distribution(torch, n, steps, tau, lid):
    """Per-step durations from the library's event log; periodogram peak of
    the series sampled at the mean step time (the paper's Fourier analysis of
    iteration times, Section 6)."""
    import workloads as W
    from paper_1309_1983_amd import Lattice
    flags = W.cavity_flags(n, n, n)
    lat = Lattice(n, n, n, tau, flags=flags, timing=steps)
    lat.set_wall_velocity(lid)
    lat.step(50)
    lat.step_times()
    lat.step(steps)
    t = lat.step_times(cap=steps).astype(np.float64)
    lat.close()
    mean, sd = float(t.mean()), float(t.std())
    x = t - t.mean()
    spec = np.abs(np.fft.rfft(x)) ** 2
    freqs = np.fft.rfftfreq(len(x), d=mean * 1e-3)

    def peak(lo, hi):
        band = np.flatnonzero((freqs >= lo) & (freqs <= hi) & (np.arange(len(freqs)) > 0))
        if len(band) == 0:
            return None, 0.0
        k = band[int(np.argmax(spec[band]))]
        return float(freqs[k]), float(np.sqrt(spec[k] * 2) / len(x))

    f_all, a_all = peak(0.0, float(freqs[-1]))
    f_low, a_low = peak(1.0, 100.0)    # the band of the paper's ~11 Hz component
    return {
        "steps": int(len(t)), "mean_ms": mean, "std_ms": sd,
        "p50_ms": float(np.percentile(t, 50)), "p99_ms": float(np.percentile(t, 99)),
        "max_ms": float(t.max()), "spikes_gt_mean_5sd": int(np.sum(t > mean + 5 * sd)),
        "even_step_mean_ms": float(t[0::2].mean()), "odd_step_mean_ms": float(t[1::2].mean()),
        "fft_peak_hz": f_all, "fft_peak_amp_ms": a_all,
        "fft_peak_amp_over_std": a_all / sd if sd > 0 else None,
        "fft_peak_1_100hz": f_low, "fft_peak_1_100hz_amp_ms": a_low,
        "fft_peak_1_100hz_amp_over_std": a_low / sd if sd > 0 else None,
    }


def adjoint_rate(torch, n, T, K, tau):
    """Reverse sweep (segment recompute + reverse steps) of a T-step rollout
    of the per-point-force duct, in MLUPS = points * T / time."""
    import workloads as W
    from paper_1309_1983_amd import Lattice
    flags = W.duct_flags(n, n, n)
    N = flags.size
    lat = Lattice(n, n, n, tau, flags=flags)
    F = torch.from_numpy(W.random_force_field(N, 1, 1e-5).astype(np.float32)).cuda()
    lat.set_force(F)
    lat.forward_checkpointed(T, K)
    g = torch.full((3, N), 1e-3, device="cuda")
    lat.adjoint(g)  # warm (allocates the adjoint buffers)
    lat.forward_checkpointed(T, K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.adjoint(g)   # synchronises before returning
    dt = time.perf_counter() - t0
    gb = lat.device_bytes() / 1e9
    lat.close()
    return N * T / dt / 1e6, gb


def config_rates(torch, steps):
    """Throughput of the other workload configurations: the 32^3 Taylor-Green
    box (cache-resident, so no roofline), the 128x128x256 sphere duct in the
    three storages, two-array, and in FP32 and FP16 offsets in place (all
    points and fluid points only), and the 512^3 cavity in FP32 two-array and
    FP16-offset in-place form."""
    import workloads as W
    from paper_1309_1983_amd import Lattice
    out = {}
    lat = Lattice(32, 32, 32, 0.8)
    u0 = torch.from_numpy(W.taylor_green_velocity(32, 32, 32, 0.05).astype(np.float32))
    lat.init_equilibrium(None, u0)
    lat.step(20)
    m = time_steps(lat, max(steps, 1000), torch)
    lat.close()
    out["tgv32_f32_ab"] = {"mlups": round(32 ** 3 / m / 1e3, 1), "ms_per_step": round(m, 5),
                           "note": "5 MB state, cache-resident and launch-bound: no roofline"}
    flags = W.sphere_duct_flags(128, 128, 256, seed=20130909, solid_fraction=0.10)
    N = flags.size
    nfl = int(np.count_nonzero(flags == 0))
    for storage, pattern in (("f32", "ab"), ("f16", "ab"), ("bf16", "ab"), ("f32", "aa"), ("f16", "aa")):
        lat = Lattice(128, 128, 256, 0.7, flags=flags, storage=storage, pattern=pattern)
        lat.set_force((0.0, 0.0, 1e-6))
        lat.step(20)
        m = time_steps(lat, steps, torch)
        lat.close()
        bpp = BYTES_PER_POINT[storage]
        out[f"spheres128x128x256_{storage}_{pattern}"] = {
            "mlups": round(N / m / 1e3, 1), "fluid_mlups": round(nfl / m / 1e3, 1),
            "ms_per_step": round(m, 5), "gbs": round(bpp * N / m / 1e6, 1),
            "frac": round(bpp * N / m / 1e6 / HBM_PEAK_GBS, 4), "fluid_fraction": round(nfl / N, 4)}
    for storage, pattern in (("f32", "ab"), ("f16", "aa")):
        lat = cavity_lattice(512, storage, pattern, 0.55, 0.05)
        lat.step(4)
        m = time_steps(lat, max(100, steps // 5), torch)
        lat.close()
        torch.cuda.empty_cache()
        bpp = BYTES_PER_POINT[storage]
        N = 512 ** 3
        out[f"cavity512_{storage}_{pattern}"] = {
            "mlups": round(N / m / 1e3, 1), "ms_per_step": round(m, 5), "gbs": round(bpp * N / m / 1e6, 1),
            "frac": round(bpp * N / m / 1e6 / HBM_PEAK_GBS, 4)}
    return out


def _time_ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def access_study(torch, n=256):
    """Section 4.3 on MI355X: aligned vs misaligned reads and writes over 19
    vectors of n^3 floats (the pull reads misaligned, the push writes
    misaligned), offset-by-one row propagation done directly, through LDS
    or with DPP lane shifts, and the push vs pull iterations."""
    import workloads as W
    from paper_1309_1983_amd import study
    N = n ** 3
    out = {"vectors": 19, "elements_per_vector": N}
    src = torch.rand(19, N, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.empty(N, device="cuda")
    rw = {}
    for width in (1, 4):
        for mode, roff, woff in (("copy", 0, 0), ("copy", 1, 0), ("copy", 0, 1), ("read", 0, 0),
                                 ("read", 1, 0), ("write", 0, 0), ("write", 0, 1)):
            ms = _time_ms(torch, lambda: study.stream(mode, src, dst, sink, N, 19, roff, woff, width), 10)
            moved = 19 * (N - 1) * 4 * (2 if mode == "copy" else 1) + ((N - 1) * 4 if mode == "read" else 0)
            key = f"{mode}_r{roff}w{woff}_x{width}"
            rw[key] = round(moved / (ms * 1e-3) / 1e9, 1)
            log(f"study {key}: {rw[key]} GB/s")
    out["read_write_gbs"] = rw
    rows = 19 * N // n
    sh = {}
    a, b = src.view(-1)[: rows * n], dst.view(-1)[: rows * n]
    for method in ("direct", "direct4", "lds", "dpp"):
        ms = _time_ms(torch, lambda: study.shift(a, b, n, rows, method), 10)
        sh[method] = round(2 * rows * n * 4 / (ms * 1e-3) / 1e9, 1)
        log(f"study shift {method}: {sh[method]} GB/s")
    out["offset_by_one_gbs"] = sh
    del src, dst
    torch.cuda.empty_cache()
    flags = torch.from_numpy((W.cavity_flags(n, n, n) != 0).astype(np.uint8)).cuda()
    fa = torch.full((19, N), 1.0 / 36, device="cuda")
    fb = fa.clone()
    pp = {}
    for scheme in ("pull", "push"):
        ms = _time_ms(torch, lambda: study.step(fa, fb, flags, n, n, n, 0.6, scheme, 256), 20)
        pp[scheme] = {"mlups": round(N / ms / 1e3, 1), "gbs": round(152 * N / (ms * 1e-3) / 1e9, 1)}
        log(f"study {scheme} (one point per work-item): {pp[scheme]}")
    out["one_point_step"] = pp
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _oracle_steps(lat, s, budget_s, max_steps):
    steps, t0 = 0, time.perf_counter()
    while True:
        s = lat.step(s)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= max_steps:
            break
    return steps, time.perf_counter() - t0


def cpu_baseline(n, tau, lid, budget_s=12.0, single_budget_s=8.0):
    """The FP64 oracle on the host: whole 256^3 cavity steps, as many as fit
    the time budget (at least one), on all the threads OpenMP takes, then on
    one thread (reported beside it as context)."""
    import oracle
    import workloads as W
    flags = W.cavity_flags(n, n, n)
    N = flags.size
    lat = oracle.Lattice(n, n, n, float(np.float32(tau)), flags=flags, uw=(float(np.float32(lid)), 0, 0))
    s = oracle.init_equilibrium(N)
    threads = oracle.num_threads()
    steps, dt = _oracle_steps(lat, s, budget_s, 50)
    oracle.set_num_threads(1)
    try:
        steps1, dt1 = _oracle_steps(lat, s, single_budget_s, 50)
    finally:
        oracle.set_num_threads(threads)
    return {"value": N * steps / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} FP64 steps of the full {n}^3 cavity ({dt:.1f} s, {_cpu_model()}, "
                      f"nproc={os.cpu_count()})",
            "one_thread": {"value": N * steps1 / dt1 / 1e6, "unit": "MLUPS",
                           "sample": f"{steps1} FP64 steps of the same cavity on 1 thread ({dt1:.1f} s)"}}


def profile_workload(torch, what, steps):
    """A few launches of one workload's kernels, for counter and trace runs
    (rocprofv3 --pmc / --kernel-trace); prints only progress."""
    import workloads as W
    from paper_1309_1983_amd import Lattice, copy_f32, study
    if what == "copy":
        n = (2 << 30) // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda").uniform_()
        b = torch.empty_like(a)
        sink = torch.empty(4, device="cuda")
        for _ in range(5):
            copy_f32(a, b)                                     # non-temporal loads and stores
        for _ in range(5):
            study.stream("copy", a, b, sink, n, 1, 0, 0, 4)    # plain 16-byte loads and stores
        torch.cuda.synchronize()
        log("copy probes done: 2 GiB read and 2 GiB written per launch")
    elif what == "cavity":
        n = 256
        for storage in ("f32", "f16", "bf16"):
            lat = cavity_lattice(n, storage, "ab", 0.6, 0.1)
            log(f"{storage}: {lat.step_kernel_name()}")
            lat.step(steps)
            if storage == "f32":
                lat.stream_only(steps)
            lat.sync()
            lat.close()
        log(f"cavity {n}^3: {steps} steps per storage, and {steps} FP32 stream-only steps")
    elif what == "spheres":
        flags = W.sphere_duct_flags(128, 128, 256, seed=20130909, solid_fraction=0.10)
        for storage, pattern in (("f32", "ab"), ("f16", "ab"), ("bf16", "ab"), ("f32", "aa"), ("f16", "aa")):
            lat = Lattice(128, 128, 256, 0.7, flags=flags, storage=storage, pattern=pattern)
            lat.set_force((0.0, 0.0, 1e-6))
            log(f"{storage} {pattern}: {lat.step_kernel_name()}")
            lat.step(steps)
            lat.sync()
            lat.close()
        log(f"sphere duct 128x128x256: {steps} steps per storage and pattern")
    elif what == "adjoint":
        n, T, K = 256, 8, 4
        flags = W.duct_flags(n, n, n)
        N = flags.size
        lat = Lattice(n, n, n, 0.7, flags=flags)
        lat.set_force(torch.from_numpy(W.random_force_field(N, 1, 1e-5).astype(np.float32)).cuda())
        lat.forward_checkpointed(T, K)
        lat.adjoint(torch.full((3, N), 1e-3, device="cuda"))
        lat.close()
        log(f"adjoint {n}^3 duct: T = {T}, K = {K}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--block", type=int, nargs=2, default=None)
    ap.add_argument("--sweep", action="store_true", help="work-group shape sweep (stderr)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--timing-steps", type=int, default=10000)
    ap.add_argument("--study", action="store_true",
                    help="run the memory-access study (Section 4.3 experiments) instead")
    ap.add_argument("--cavity", action="store_true",
                    help="run the cavity validation (Section 5: Re 100, 400, 1000 with on-site "
                         "walls, Eq. (8) scaling, doubled resolutions) instead")
    ap.add_argument("--profile", choices=["cavity", "spheres", "adjoint", "copy"], default=None,
                    help="run a few launches of one workload's kernels for rocprofv3 and exit: "
                         "cavity (256^3 FP32/FP16/BF16 steps and the FP32 stream-only step), spheres "
                         "(sphere duct, every storage, AB and AA), adjoint (256^3 reverse sweep, T=8, "
                         "K=4), copy (the copy probe with and without load hints, 2 GiB)")
    ap.add_argument("--pmc-summary", metavar="DIR", default=None,
                    help="summarise the rocprofv3 counter passes under DIR (<pass>_<workload> "
                         "folders from --profile runs) into profiles/pmc_traffic_*.json and exit; "
                         "runs on the host, no GPU")
    ap.add_argument("--copy-only", action="store_true",
                    help="run only the copy probe (2 GiB float32, 20 launches): counter calibration")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path is "
              "single-GPU; multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    if args.pmc_summary:
        for path in pmc_summary(args.pmc_summary, os.path.join(ROOT, "profiles")):
            print(path)
        return

    import torch
    import paper_1309_1983_amd
    paper_1309_1983_amd.lib()
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"

    if args.study:
        print(json.dumps({"study": access_study(torch, args.n)}), flush=True)
        return

    if args.cavity:
        from paper_1309_1983_amd import cavity
        out = cavity.validation(log=sys.stderr)
        summary = {}
        for Re, v in out.items():
            summary[str(Re)] = {
                "runs": [{k: r.as_dict()[k] for k in ("L", "tau", "u_lid", "steps", "converged", "residual",
                                                      "finite", "seconds", "glups")} for r in v["runs"]],
                "fixed": v["fixed"],
                "max_profile_differences": v["differences"], "observed_orders": v["orders"],
                "rms_profile_differences": v["rms_differences"], "rms_orders": v["rms_orders"],
                "finest": {k: v["runs"][-1].as_dict()[k] for k in ("L", "y", "ux", "x", "uy")},
            }
        print(json.dumps({"cavity_validation": summary}), flush=True)
        return

    if args.profile:
        profile_workload(torch, args.profile, max(1, min(args.steps, 20)))
        return

    if args.copy_only:
        cc = copy_ceiling(torch)
        print(json.dumps({"copy_gbs": round(cc, 1), "bytes_per_launch": 2 * (2 << 30)}), flush=True)
        return

    n, tau, lid = args.n, 0.6, 0.1
    N = n ** 3
    workload = f"cavity{n}"
    log(f"device {torch.cuda.get_device_name(0)}; workload {workload}")

    sweep = None
    if args.sweep:
        # work-group shapes (Section 6 sweeps 64..1024 threads per block): the
        # four-point kernel (up to 256 work-items = 1024 points per group) and
        # the one-point kernel (up to 1024 work-items)
        sweep = []
        shapes = [(4, bx, by) for bx, by in [(16, 1), (32, 1), (64, 1), (128, 1), (256, 1), (64, 2),
                                             (64, 4), (128, 2), (32, 8)]]
        shapes += [(1, bx, by) for bx, by in [(64, 1), (128, 1), (256, 1), (512, 1), (1024, 1), (256, 4)]]
        for cpl, bx, by in shapes:
            lat = cavity_lattice(n, "f32", "ab", tau, lid, block=(bx, by), cells_per_lane=cpl)
            lat.step(args.warmup)
            ms = time_steps(lat, max(200, args.steps // 2), torch)
            lat.close()
            sweep.append({"points_per_work_item": cpl, "block": [bx, by], "points_per_group": cpl * bx * by,
                          "ms_per_step": round(ms, 5), "mlups": round(N / ms / 1e3, 1),
                          "gbs": round(BYTES_PER_POINT["f32"] * N / ms / 1e6, 1)})
            log(f"sweep {cpl} point(s) per work-item, block {bx}x{by}: {ms:.4f} ms/step, "
                f"{N / ms / 1e3:.0f} MLUPS, {BYTES_PER_POINT['f32'] * N / ms / 1e6:.0f} GB/s")

    # ---- headline: FP32 two-array step ----
    lat = cavity_lattice(n, "f32", "ab", tau, lid, block=args.block)
    kernel_name = lat.step_kernel_name()     # the kernel the library's dispatch launches
    lat.step(args.warmup)
    torch.cuda.synchronize()
    log(f"timing {args.steps} FP32 AB steps ({kernel_name})")
    ms = time_steps(lat, args.steps, torch)
    lat.check_finite()
    lat.close()
    mlups = N / ms / 1e3
    achieved = BYTES_PER_POINT["f32"] * N / (ms * 1e-3) / 1e9
    traffic = load_traffic(workload, kernel_name)
    line = {
        "metric": "MLUPS and % HBM roofline, D3Q19 FP32 256^3; FP16-storage and adjoint MLUPS",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"D3Q19 BGK lid-driven cavity {n}^3, FP32 two-array pull step, "
                               f"halfway bounce-back walls, lid 0.1 in x, tau 0.6, from rest",
                   "nx": n, "ny": n, "nz": n, "storage": "f32", "pattern": "ab",
                   "block": list(args.block) if args.block else "default"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_point": BYTES_PER_POINT["f32"],
                     "kernel": kernel_name},
    }
    # the paper's own figure, on other hardware: context only, not vs_baseline
    line["paper_context"] = {"mlups": 1036.41, "device": "Tesla K20c (measured 157.89 GB/s)",
                             "config": "FP32 D3Q19, 192^3, block 64 (Table 2)"}
    log(f"FP32 AB: {ms:.4f} ms/step, {mlups:.0f} MLUPS, {achieved:.0f} GB/s "
        f"({100 * achieved / HBM_PEAK_GBS:.1f}% of 8 TB/s)")
    if sweep is not None:
        line["sweep"] = sweep

    if not args.no_extra:
        extra = {}
        cc = copy_ceiling(torch)
        extra["copy_ceiling_gbs"] = round(cc, 1)
        line["roofline"]["frac_of_copy_ceiling"] = round(achieved / cc, 4)
        log(f"copy ceiling {cc:.0f} GB/s")
        # the access pattern's own ceiling: the same gather and stores with no
        # collision (lbm_debug_stream_only), and the 19 planes without shifts
        lat = cavity_lattice(n, "f32", "ab", tau, lid, block=args.block)
        lat.stream_only(args.warmup)
        m = time_steps(lat, args.steps, torch, stream_only=True)
        lat.close()
        gbs = BYTES_PER_POINT["f32"] * N / (m * 1e-3) / 1e9
        extra["stream_only_f32_ab"] = {"mlups": round(N / m / 1e3, 1), "ms_per_step": round(m, 5),
                                       "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                       "step_time_over_stream_only": round(ms / m, 4)}
        log(f"stream only (no collision): {m:.4f} ms/step, {gbs:.0f} GB/s; step/stream-only = {ms / m:.4f}")
        extra["pattern_ceilings"] = pattern_ceilings(torch, n) if n % 4 == 0 else None
        log(f"pattern ceilings: {extra['pattern_ceilings']}")
        for storage, pattern, cpl in (("f16", "ab", 0), ("bf16", "ab", 0), ("f16", "ab", 4),
                                      ("bf16", "ab", 4), ("f16", "aa", 0), ("bf16", "aa", 0),
                                      ("f32", "aa", 0)):
            lat = cavity_lattice(n, storage, pattern, tau, lid, cells_per_lane=cpl)
            lat.step(args.warmup)
            m = time_steps(lat, args.steps, torch)
            lat.close()
            bpp = BYTES_PER_POINT[storage]
            gbs = bpp * N / (m * 1e-3) / 1e9
            key = f"{storage}_{pattern}" + (f"_w{cpl}" if cpl else "")
            extra[key] = {"mlups": round(N / m / 1e3, 1), "ms_per_step": round(m, 5),
                          "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                          "bytes_per_point": bpp}
            log(f"{key}: {m:.4f} ms/step, {N / m / 1e3:.0f} MLUPS, {gbs:.0f} GB/s")
        # the cavity closed by on-site velocity walls (the paper's validation boundaries)
        lat = cavity_lattice(n, "f32", "ab", tau, lid, onsite=True)
        lat.step(args.warmup)
        m = time_steps(lat, args.steps, torch)
        lat.check_finite()
        lat.close()
        gbs = BYTES_PER_POINT["f32"] * N / (m * 1e-3) / 1e9
        extra["f32_ab_onsite_walls"] = {"mlups": round(N / m / 1e3, 1), "ms_per_step": round(m, 5),
                                        "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                        "bytes_per_point": BYTES_PER_POINT["f32"]}
        log(f"f32_ab on-site walls: {m:.4f} ms/step, {N / m / 1e3:.0f} MLUPS, {gbs:.0f} GB/s")
        # the step with rho and u stored every step (four extra stores per point)
        lat = cavity_lattice(n, "f32", "ab", tau, lid)
        lat.step(args.warmup)
        rho = torch.empty(N, device="cuda")
        u = torch.empty(3, N, device="cuda")
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        from paper_1309_1983_amd import _abi
        import ctypes
        for _ in range(args.steps):
            _abi.call("lbm_step_macros", lat._h, 1, ctypes.c_void_p(rho.data_ptr()),
                      ctypes.c_void_p(u.data_ptr()))
        e1.record(lat.stream)
        torch.cuda.synchronize()
        m = e0.elapsed_time(e1) / args.steps
        lat.close()
        bpp = BYTES_PER_POINT["f32"] + MACROS_BYTES
        gbs = bpp * N / (m * 1e-3) / 1e9
        extra["f32_ab_macros_every_step"] = {"mlups": round(N / m / 1e3, 1), "ms_per_step": round(m, 5),
                                             "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                             "bytes_per_point": bpp}
        log(f"f32_ab with rho,u every step: {m:.4f} ms/step, {N / m / 1e3:.0f} MLUPS, {gbs:.0f} GB/s")
        for key, an, T, K in (("adjoint", n, 200, 50), ("adjoint64", 64, 200, 20)):
            try:
                ar, gb = adjoint_rate(torch, an, T=T, K=K, tau=0.7)
                gbs = ar * 1e6 * ADJOINT_BYTES_PER_POINT / 1e9
                extra[key] = {"mlups": round(ar, 1), "T": T, "K": K, "device_gb": round(gb, 2),
                              "workload": f"duct {an}^3, per-point force, tau 0.7",
                              "bytes_per_point": ADJOINT_BYTES_PER_POINT, "gbs_alg": round(gbs, 1),
                              "frac": round(gbs / HBM_PEAK_GBS, 4)}
                if an <= 64:
                    extra[key]["note"] = "20 MB states: largely cache-resident, no roofline claim"
                log(f"{key}: {ar:.0f} MLUPS (reverse sweep incl. recompute), {gb:.1f} GB on device")
            except Exception as e:  # noqa: BLE001
                extra[key] = {"error": str(e)}
        log("other workload configurations")
        extra["configs"] = config_rates(torch, args.steps)
        for k, v in extra["configs"].items():
            log(f"{k}: {v}")
        if args.timing_steps > 0:
            log(f"per-step timing log over {args.timing_steps} steps")
            extra["step_time"] = step_time_distribution(torch, n, args.timing_steps, tau, lid)
        line["extra"] = extra

    if not args.no_cpu:
        log("CPU baseline (FP64 oracle)")
        line["cpu_baseline"] = cpu_baseline(n, tau, lid)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
