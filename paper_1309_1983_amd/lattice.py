"""Python handle over the C ABI: a D3Q19 lattice living in device memory.

Every method marshals arguments and calls one entry point of liblbm_hip.so;
torch supplies device tensors for inputs and outputs and the HIP stream the
library launches on. Nothing here computes lattice Boltzmann arithmetic.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _abi

Q = 19


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


class Lattice:
    """nx*ny*nz D3Q19 lattice (index c = (z*ny + y)*nx + x, populations [19][N]).

    flags: uint8 per point (0 fluid, 1 wall, 2 moving wall, 3 on-site velocity
    node at rest, 4 on-site node moving with the wall velocity) as numpy / torch /
    None (all fluid). storage: 'f32' | 'f16' | 'bf16' (16-bit offsets).
    pattern: 'ab' (two arrays) | 'aa' (one array, in place).
    """

    GATHER_MODES = {"auto": 0, "flags_first": 1, "early": 2}

    def __init__(self, nx, ny, nz, tau, flags=None, storage="f32", pattern="ab", block=None,
                 timing=0, check_interval=0, device=None, stream=None, cells_per_lane=0,
                 gather_mode="auto", groups_per_cu=0, torch_buffers=False):
        if not torch.cuda.is_available():
            raise RuntimeError("Lattice needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.N = self.nx * self.ny * self.nz
        self.storage, self.pattern = storage, pattern
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        opt = _abi.lbm_options()
        _abi.lib().lbm_options_default(ctypes.byref(opt))
        opt.storage = _abi.STORAGE[storage]
        opt.pattern = _abi.PATTERN[pattern]
        opt.hip_stream = ctypes.c_void_p(stream.cuda_stream)
        if block is not None:
            opt.block_x, opt.block_y = int(block[0]), int(block[1])
        opt.timing_capacity = int(timing)
        opt.check_interval = int(check_interval)
        opt.device = self.device.index
        opt.cells_per_lane = int(cells_per_lane)
        opt.gather_mode = self.GATHER_MODES[gather_mode]
        opt.groups_per_cu = int(groups_per_cu)
        # torch_buffers: the population arrays, the adjoint workspace and the
        # checkpoint store are torch allocations handed to the library
        self.torch_buffers = bool(torch_buffers)
        self._bufs = {}
        if self.torch_buffers:
            sizes = _abi.lbm_buffer_sizes()
            _abi.call("lbm_query_buffer_sizes", self.nx, self.ny, self.nz, ctypes.byref(opt),
                      ctypes.byref(sizes))
            self._sizes = sizes
            pops = [self._device_buffer(sizes.population_bytes) for _ in range(sizes.population_arrays)]
            self._bufs["populations"] = pops
            for b, t in enumerate(pops):
                opt.population_dev[b] = t.data_ptr()
        fl = None
        if flags is not None:
            fl = np.ascontiguousarray(
                flags.cpu().numpy() if isinstance(flags, torch.Tensor) else flags, dtype=np.uint8)
            if fl.size != self.N:
                raise ValueError(f"flags has {fl.size} entries, lattice has {self.N}")
        self._flags = fl
        h = ctypes.c_void_p()
        _abi.call("lbm_create_ex", self.nx, self.ny, self.nz, ctypes.c_float(tau),
                  fl.ctypes.data_as(ctypes.c_void_p) if fl is not None else None,
                  ctypes.byref(opt), ctypes.byref(h))
        self._h = h
        self.tau = float(np.float32(tau))
        if self.torch_buffers and storage == "f32" and pattern == "ab":
            adj = self._device_buffer(self._sizes.adjoint_bytes)
            _abi.call("lbm_set_adjoint_buffer", self._h, _ptr(adj), ctypes.c_size_t(adj.numel()))
            self._bufs["adjoint"] = adj

    def _device_buffer(self, nbytes):
        """A torch byte buffer on the lattice's device, 256-byte aligned."""
        t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        if t.data_ptr() % 256:
            raise RuntimeError("torch returned a buffer that is not 256-byte aligned")
        return t

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _abi.lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- parameters ---------------------------------------------------------
    def set_tau(self, tau):
        _abi.call("lbm_set_tau", self._h, ctypes.c_float(tau))
        self.tau = float(np.float32(tau))

    def set_wall_velocity(self, ux, uy=0.0, uz=0.0):
        _abi.call("lbm_set_wall_velocity", self._h, ctypes.c_float(ux), ctypes.c_float(uy),
                  ctypes.c_float(uz))

    def set_force(self, force):
        """force: 3-sequence (uniform), torch tensor [3, N] (field) or None."""
        if force is None:
            _abi.call("lbm_set_force_field", self._h, None)
            _abi.call("lbm_set_force_uniform", self._h, 0.0, 0.0, 0.0)
        elif isinstance(force, torch.Tensor) and force.numel() == 3 * self.N:
            F = self._dev_f32(force, (3, self.N))
            _abi.call("lbm_set_force_field", self._h, _ptr(F))
            self._force_keep = F
        else:
            fx, fy, fz = (float(v) for v in force)
            _abi.call("lbm_set_force_uniform", self._h, ctypes.c_float(fx), ctypes.c_float(fy),
                      ctypes.c_float(fz))

    def set_stream(self, stream):
        _abi.call("lbm_set_stream", self._h, ctypes.c_void_p(stream.cuda_stream))
        self.stream = stream

    # -- state --------------------------------------------------------------
    def _dev_f32(self, t, shape):
        t = torch.as_tensor(t)
        t = t.to(device=self.device, dtype=torch.float32).reshape(shape).contiguous()
        return t

    def init_equilibrium(self, rho=None, u=None):
        r = self._dev_f32(rho, (self.N,)) if rho is not None else None
        v = self._dev_f32(u, (3, self.N)) if u is not None else None
        _abi.call("lbm_init_equilibrium", self._h, _ptr(r), _ptr(v))
        self._keep = (r, v)

    def step(self, n=1):
        _abi.call("lbm_step", self._h, int(n))

    def step_macros(self, n=1):
        """n steps; the last one also returns its in-step (rho [N], u [3, N])."""
        rho = torch.empty(self.N, dtype=torch.float32, device=self.device)
        u = torch.empty(3, self.N, dtype=torch.float32, device=self.device)
        _abi.call("lbm_step_macros", self._h, int(n), _ptr(rho), _ptr(u))
        return rho, u

    def stream_only(self, n=1):
        _abi.call("lbm_debug_stream_only", self._h, int(n))

    def macros(self):
        rho = torch.empty(self.N, dtype=torch.float32, device=self.device)
        u = torch.empty(3, self.N, dtype=torch.float32, device=self.device)
        _abi.call("lbm_macros", self._h, _ptr(rho), _ptr(u))
        return rho, u

    def populations(self):
        f = torch.empty(Q, self.N, dtype=torch.float32, device=self.device)
        _abi.call("lbm_get_populations", self._h, _ptr(f))
        return f

    def set_populations(self, f):
        F = self._dev_f32(f, (Q, self.N))
        _abi.call("lbm_set_populations", self._h, _ptr(F))
        self._keep = F

    def check_finite(self):
        _abi.call("lbm_check_finite", self._h)

    def sync(self):
        _abi.call("lbm_sync", self._h)

    def step_times(self, cap=1 << 20):
        buf = (ctypes.c_float * cap)()
        n = ctypes.c_int(0)
        _abi.call("lbm_step_times", self._h, buf, cap, ctypes.byref(n))
        return np.frombuffer(buf, dtype=np.float32, count=n.value).copy()

    def step_kernel_name(self):
        """Demangled name of the kernel the next step() launches."""
        buf = ctypes.create_string_buffer(512)
        _abi.call("lbm_step_kernel_name", self._h, buf, ctypes.c_size_t(len(buf)))
        return buf.value.decode()

    def device_bytes(self):
        return int(_abi.lib().lbm_device_bytes(self._h))

    # -- adjoint ------------------------------------------------------------
    def forward_checkpointed(self, T, K):
        if self.torch_buffers:
            need = int(_abi.lib().lbm_trajectory_bytes(self.nx, self.ny, self.nz, int(T), int(K)))
            cur = self._bufs.get("trajectory")
            if cur is None or cur.numel() < need:
                # the library stops using the old buffer before returning
                self._bufs["trajectory"] = None
                traj = self._device_buffer(max(need, 256))
                _abi.call("lbm_set_trajectory_buffer", self._h, _ptr(traj), ctypes.c_size_t(traj.numel()))
                self._bufs["trajectory"] = traj
        _abi.call("lbm_forward_checkpointed", self._h, int(T), int(K))

    def adjoint(self, dL_du):
        """(grad_F [3, N], grad_tau) for the trajectory of forward_checkpointed."""
        g = self._dev_f32(dL_du, (3, self.N))
        gF = torch.empty(3, self.N, dtype=torch.float32, device=self.device)
        gt = ctypes.c_double(0.0)
        _abi.call("lbm_adjoint", self._h, _ptr(g), _ptr(gF), ctypes.byref(gt))
        return gF, gt.value


def copy_f32(src: torch.Tensor, dst: torch.Tensor, stream=None):
    """dst[:] = src[:] with the library's copy probe kernel (float32, device)."""
    assert src.dtype == torch.float32 and dst.dtype == torch.float32
    assert src.is_contiguous() and dst.is_contiguous() and src.numel() <= dst.numel()
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    _abi.call("lbm_copy_f32", _ptr(src), _ptr(dst), ctypes.c_size_t(src.numel()),
              ctypes.c_void_p(s.cuda_stream))
