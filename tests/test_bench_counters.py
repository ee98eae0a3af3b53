"""Host-side arithmetic of the benchmark's counter summaries (no GPU): the
copy-probe calibration, the exact EA request bytes, the per-kernel
algorithmic bytes, and the source-hash guard on the reported traffic."""
import csv
import json
import os

import pytest

import bench

STEP = ("void lbmk::k_step_abv<d3q19::StF32, 0, true, 4, false, false, false, false>"
        "(d3q19::StF32::bits_t const*, d3q19::StF32::bits_t*, unsigned char const*, unsigned int const*, "
        "unsigned int const*, float const*, lbmk::StepArgs, float*, float*)")
ADJ = "void lbmk::k_adj_stepv<2, false, 2>(float const*, float const*, float*, float*, double*)"
COPY = "lbmk::k_copy(float const*, float*, unsigned long)"


def _write_pass(root, name, rows):
    d = root / name
    d.mkdir()
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for k, (kernel, counter, value) in enumerate(rows):
            w.writerow([k, kernel, counter, value])


def _fake_passes(root):
    """Counter passes as gfx950 reports them: FETCH_SIZE counts a 128-byte read
    request as 64 bytes (KiB), WRITE_SIZE is exact, all reads are 128-byte
    requests and all writes 64-byte ones."""
    two_gib = 2 << 30
    step_rd, step_wr = 1_327_800_064, 1_255_280_640     # bytes, multiples of 128 / 64
    adj_rd, adj_wr = 3_212_300_288, 1_468_500_032
    for w, kernels in (("cavity", [(STEP, step_rd, step_wr)]), ("spheres", [(STEP, step_rd, step_wr)]),
                       ("adjoint", [(ADJ, adj_rd, adj_wr)]), ("copy", [(COPY, two_gib, two_gib)])):
        _write_pass(root, f"fetch_{w}", [(k, "FETCH_SIZE", rd / 2 / 1024) for k, rd, _ in kernels] * 2)
        _write_pass(root, f"write_{w}", [(k, "WRITE_SIZE", wr / 1024) for k, _, wr in kernels] * 2)
        _write_pass(root, f"rdreq_{w}", [r for k, rd, _ in kernels for r in (
            (k, "TCC_EA0_RDREQ_32B_sum", 0), (k, "TCC_EA0_RDREQ_64B_sum", 0),
            (k, "TCC_EA0_RDREQ_128B_sum", rd // 128), (k, "TCC_EA0_RDREQ_sum", rd // 128))])
        _write_pass(root, f"wrreq_{w}", [r for k, _, wr in kernels for r in (
            (k, "TCC_EA0_WRREQ_sum", wr // 64), (k, "TCC_EA0_WRREQ_64B_sum", wr // 64))])
        _write_pass(root, f"hit_{w}", [r for k, _, _ in kernels for r in (
            (k, "TCC_HIT_sum", 1.0), (k, "TCC_MISS_sum", 3.0))])
    return step_rd, step_wr, adj_rd, adj_wr


def test_kernel_key_drops_the_parameter_list_only():
    assert bench._kernel_key(STEP) == "lbmk::k_step_abv<d3q19::StF32, 0, true, 4, false, false, false, false>"
    assert bench._kernel_key("(anonymous namespace)::k_planes<1>(float const*, float*)") == \
        "(anonymous namespace)::k_planes<1>"
    assert bench._kernel_key("lbmk::k_mark_near_wall") == "lbmk::k_mark_near_wall"


def test_algorithmic_bytes_per_point():
    assert bench._algorithmic_bytes_per_point("lbmk::k_step_abv<d3q19::StF32, 0, true, 4, false, false, false, false>") == 152
    assert bench._algorithmic_bytes_per_point("lbmk::k_step_abv<d3q19::StBF16, 1, true, 4, false, false, false, false>") == 76
    assert bench._algorithmic_bytes_per_point("lbmk::k_step_abv<d3q19::StF32, 2, true, 4, false, false, false, false>") == 164
    assert bench._algorithmic_bytes_per_point("lbmk::k_step_aa0<d3q19::StF16, 1, true, false>") == 76
    assert bench._algorithmic_bytes_per_point("lbmk::k_adj_stepv<2, false, 2>") == 264
    assert bench._algorithmic_bytes_per_point("lbmk::k_init_eq<d3q19::StF32>") is None


def test_pmc_summary_calibrates_and_counts_exactly(tmp_path):
    (tmp_path / "pmc").mkdir()
    step_rd, step_wr, adj_rd, adj_wr = _fake_passes(tmp_path / "pmc")
    out = tmp_path / "profiles"
    out.mkdir()
    paths = bench.pmc_summary(str(tmp_path / "pmc"), str(out))
    assert sorted(os.path.basename(p) for p in paths) == [
        "pmc_traffic_adjoint256.json", "pmc_traffic_cavity256.json", "pmc_traffic_spheres128x128x256.json"]
    cav = json.load(open(out / "pmc_traffic_cavity256.json"))
    assert cav["calibration"]["fetch_factor"] == pytest.approx(2.0, rel=1e-9)
    assert cav["calibration"]["write_factor"] == pytest.approx(1.0, rel=1e-9)
    (k,) = cav["kernels"]
    assert k["dispatches"] == 2
    assert k["hbm_read_bytes"] == step_rd and k["hbm_write_bytes"] == step_wr
    assert k["ea_read_bytes_from_request_sizes"] == step_rd
    assert k["ea_write_bytes_from_request_sizes"] == step_wr
    assert k["algorithmic_bytes_per_launch"] == 152 * 256 ** 3
    assert k["traffic_over_algorithmic"] == pytest.approx((step_rd + step_wr) / (152 * 256 ** 3), abs=1e-4)
    assert k["l2_hit_rate"] == pytest.approx(0.25)
    assert cav["kernel_source_hash"] == bench.kernel_source_hash()
    adj = json.load(open(out / "pmc_traffic_adjoint256.json"))
    (k,) = adj["kernels"]
    assert k["hbm_bytes_per_launch"] == adj_rd + adj_wr
    assert k["algorithmic_bytes_per_launch"] == 264 * 256 ** 3


def test_traffic_is_reported_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    doc = {"kernel_source_hash": bench.kernel_source_hash(),
           "kernels": [{"kernel": bench._kernel_key(STEP), "hbm_bytes_per_launch": 123}]}
    (prof / "pmc_traffic_cavity256.json").write_text(json.dumps(doc))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: doc["kernel_source_hash"])
    assert bench.load_traffic("cavity256", STEP) == 123
    assert bench.load_traffic("cavity256", ADJ) is None            # no entry for that kernel
    assert bench.load_traffic("spheres128x128x256", STEP) is None  # no file
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("cavity256", STEP) is None            # counters of another source
