"""Host-side tests of the C ABI: the library loads, exports every entry point
that include/lbm.h declares, and rejects bad arguments before any HIP call
(so these run without a GPU)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
STUDY_HEADER = os.path.join(ROOT, "include", "lbm_study.h")


@pytest.fixture(scope="module")
def abi():
    from paper_1309_1983_amd import _abi
    if not os.path.exists(_abi.lib_path()):
        from paper_1309_1983_amd import build
        build.build()
    _abi.lib()
    return _abi


def _declared_functions(header=None):
    if header is None:
        return sorted(set(_declared_functions(HEADER)) | set(_declared_functions(STUDY_HEADER)))
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree(abi):
    assert _declared_functions(HEADER) == sorted(abi.EXPORTS)
    assert _declared_functions(STUDY_HEADER) == sorted(abi.STUDY_EXPORTS)


def test_library_exports_every_declared_symbol(abi):
    out = subprocess.run(["nm", "-D", "--defined-only", abi.lib_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [f for f in _declared_functions() if f not in exported]
    assert not missing, missing
    for f in _declared_functions():
        assert hasattr(abi.lib(), f)


def test_library_is_built_for_gfx950(abi):
    data = open(abi.lib_path(), "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_options_default(abi):
    opt = abi.lbm_options()
    opt.storage = 7
    abi.lib().lbm_options_default(ctypes.byref(opt))
    assert (opt.storage, opt.pattern, opt.block_x, opt.block_y) == (0, 0, 0, 0)
    assert opt.timing_capacity == 0 and opt.check_interval == 0 and opt.device == -1
    assert not opt.hip_stream


def _create(abi, nx, ny, nz, tau, flags=None, opt=None):
    h = ctypes.c_void_p()
    fp = flags.ctypes.data_as(ctypes.c_void_p) if flags is not None else None
    if opt is None:
        st = abi.lib().lbm_create(nx, ny, nz, ctypes.c_float(tau), fp, ctypes.byref(h))
    else:
        st = abi.lib().lbm_create_ex(nx, ny, nz, ctypes.c_float(tau), fp, ctypes.byref(opt),
                                     ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("dims,tau,msg", [
    ((0, 4, 4), 0.8, "positive"),
    ((4, -1, 4), 0.8, "positive"),
    ((1024, 1024, 1024), 0.8, "2^30"),
    ((8, 8, 70000), 0.8, "65535"),
    ((8, 8, 8), 0.5, "tau"),
    ((8, 8, 8), float("nan"), "tau"),
    ((8, 8, 8), 0.3, "tau"),
])
def test_create_rejects_bad_arguments(abi, dims, tau, msg):
    st, h = _create(abi, *dims, tau)
    assert st == abi.LBM_ERR_INVALID
    assert not h.value
    assert msg in abi.last_error()


def test_create_rejects_bad_flags_and_options(abi):
    flags = np.zeros(64, dtype=np.uint8)
    flags[17] = 5
    st, _ = _create(abi, 4, 4, 4, 0.8, flags)
    assert st == abi.LBM_ERR_INVALID and "flag value 5" in abi.last_error()
    for field, value in (("storage", 3), ("pattern", 2), ("block_x", 2048), ("block_y", -1),
                         ("timing_capacity", -5)):
        opt = abi.lbm_options()
        abi.lib().lbm_options_default(ctypes.byref(opt))
        setattr(opt, field, value)
        if field == "block_y":
            opt.block_x = 64
        st, _ = _create(abi, 8, 8, 8, 0.8, None, opt)
        assert st == abi.LBM_ERR_INVALID, field
    st = abi.lib().lbm_create(4, 4, 4, ctypes.c_float(0.8), None, None)
    assert st == abi.LBM_ERR_INVALID


def test_create_rejects_bad_modes_and_caller_buffers(abi):
    """Caller-owned population arrays and the launch-mode options are
    validated before any HIP call."""
    def opt_with(**kw):
        opt = abi.lbm_options()
        abi.lib().lbm_options_default(ctypes.byref(opt))
        for k, v in kw.items():
            if k == "population_dev":
                opt.population_dev[0], opt.population_dev[1] = v
            else:
                setattr(opt, k, v)
        return opt
    cases = [
        (dict(gather_mode=-1), "gather_mode"),
        (dict(groups_per_cu=-2), "groups_per_cu"),
        (dict(groups_per_cu=65), "groups_per_cu"),
        (dict(population_dev=(4096, None)), "population_dev[1] is NULL"),
        (dict(population_dev=(4096 + 64, 8192)), "256-byte aligned"),
        (dict(population_dev=(4096, 4096)), "different"),
        (dict(pattern=1, population_dev=(4096, 8192)), "must be NULL for the AA"),
    ]
    for kw, msg in cases:
        st, h = _create(abi, 8, 8, 8, 0.8, None, opt_with(**kw))
        assert st == abi.LBM_ERR_INVALID and not h.value, kw
        assert msg in abi.last_error(), (kw, abi.last_error())


def test_buffer_size_queries(abi):
    """Sizes a caller needs to allocate the library's buffers itself:
    19 populations per point in 4 or 2 bytes, two arrays for AB and one for
    AA; the adjoint workspace holds two FP32 states; the checkpoint store
    ceil(T/K) + min(K, T) - 1 states."""
    L = abi.lib()
    out = abi.lbm_buffer_sizes()
    nx, ny, nz = 36, 10, 9
    N = nx * ny * nz
    assert L.lbm_query_buffer_sizes(nx, ny, nz, None, ctypes.byref(out)) == abi.LBM_OK
    r256 = lambda b: (b + 255) // 256 * 256
    assert out.population_bytes == r256(19 * N * 4) and out.population_arrays == 2
    assert out.state_bytes == 19 * N * 4
    assert out.adjoint_bytes >= 2 * r256(19 * N * 4) + 8
    opt = abi.lbm_options()
    L.lbm_options_default(ctypes.byref(opt))
    opt.storage, opt.pattern = abi.STORAGE["f16"], abi.PATTERN["aa"]
    assert L.lbm_query_buffer_sizes(nx, ny, nz, ctypes.byref(opt), ctypes.byref(out)) == abi.LBM_OK
    assert out.population_bytes == r256(19 * N * 2) and out.population_arrays == 1
    assert L.lbm_query_buffer_sizes(0, ny, nz, None, ctypes.byref(out)) == abi.LBM_ERR_INVALID
    assert L.lbm_query_buffer_sizes(nx, ny, nz, None, None) == abi.LBM_ERR_INVALID
    sb = r256(19 * N * 4)
    assert L.lbm_trajectory_bytes(nx, ny, nz, 200, 20) == (10 + 19) * sb
    assert L.lbm_trajectory_bytes(nx, ny, nz, 12, 5) == (3 + 4) * sb
    assert L.lbm_trajectory_bytes(nx, ny, nz, 0, 5) == 1 * sb
    assert L.lbm_trajectory_bytes(nx, ny, nz, 3, 10) == (1 + 2) * sb
    assert L.lbm_trajectory_bytes(nx, ny, nz, 5, 0) == 0


def test_calls_on_null_lattice(abi):
    L = abi.lib()
    assert L.lbm_step(None, 1) == abi.LBM_ERR_INVALID
    assert L.lbm_macros(None, None, None) == abi.LBM_ERR_INVALID
    assert L.lbm_set_tau(None, ctypes.c_float(0.7)) == abi.LBM_ERR_INVALID
    assert L.lbm_forward_checkpointed(None, 10, 2) == abi.LBM_ERR_INVALID
    gt = ctypes.c_double()
    assert L.lbm_adjoint(None, None, None, ctypes.byref(gt)) == abi.LBM_ERR_INVALID
    assert L.lbm_device_bytes(None) == 0
    assert L.lbm_set_trajectory_buffer(None, None, 0) == abi.LBM_ERR_INVALID
    assert L.lbm_set_adjoint_buffer(None, None, 0) == abi.LBM_ERR_INVALID
    assert L.lbm_set_stream(None, None) == abi.LBM_ERR_INVALID
    L.lbm_destroy(None)  # no-op


def test_copy_probe_rejects_null_and_misaligned_buffers(abi):
    # validated before any HIP call, so this runs without a GPU
    L = abi.lib()
    n = ctypes.c_size_t(8)
    assert L.lbm_copy_f32(None, None, n, None) == abi.LBM_ERR_INVALID
    assert L.lbm_copy_f32(ctypes.c_void_p(4096 + 4), ctypes.c_void_p(8192), n, None) == abi.LBM_ERR_INVALID
    assert "aligned" in abi.last_error()
    assert L.lbm_copy_f32(ctypes.c_void_p(4096), ctypes.c_void_p(8192 + 8), n, None) == abi.LBM_ERR_INVALID


def test_study_calls_reject_bad_arguments(abi):
    L = abi.lib()
    assert L.lbm_study_stream(0, None, None, None, 1024, 19, 0, 0, 4, None) == abi.LBM_ERR_INVALID
    assert L.lbm_study_stream(3, None, None, None, 1024, 19, 0, 0, 4, None) == abi.LBM_ERR_INVALID
    assert L.lbm_study_shift(None, None, 256, 4, 0, None) == abi.LBM_ERR_INVALID
    assert L.lbm_study_step(None, None, None, 8, 8, 8, ctypes.c_float(0.8), 0, 64, None) == abi.LBM_ERR_INVALID
    assert L.lbm_study_planes(0, None, None, None, 256, 4, 4, None) == abi.LBM_ERR_INVALID
    assert L.lbm_study_planes(3, ctypes.c_void_p(4096), ctypes.c_void_p(8192), None, 256, 4, 4, None) == abi.LBM_ERR_INVALID
    assert L.lbm_study_planes(0, ctypes.c_void_p(4096), ctypes.c_void_p(8192), None, 254, 4, 4, None) == abi.LBM_ERR_INVALID
    assert L.lbm_study_planes(0, ctypes.c_void_p(4100), ctypes.c_void_p(8192), None, 256, 4, 4, None) == abi.LBM_ERR_INVALID


def test_status_strings(abi):
    names = [abi.status_name(s) for s in range(6)]
    assert names == ["LBM_OK", "LBM_ERR_INVALID", "LBM_ERR_OOM", "LBM_ERR_DEVICE",
                     "LBM_ERR_STATE", "LBM_ERR_NONFINITE"]
    assert abi.status_name(99) == "LBM_ERR_UNKNOWN"


def test_last_error_is_per_thread(abi):
    import threading
    _create(abi, 0, 1, 1, 0.8)
    main_msg = abi.last_error()
    seen = {}

    def worker():
        seen["before"] = abi.last_error()
        _create(abi, 8, 8, 8, 0.2)
        seen["after"] = abi.last_error()

    t = threading.Thread(target=worker)
    t.start()
    t.join()
    assert seen["before"] == ""
    assert "tau" in seen["after"]
    assert abi.last_error() == main_msg


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1309_1983_amd import _abi
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "_LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError, match="no CPU fallback"):
        _abi.lib()
