"""Plain FP64 CPU oracle for the D3Q19 BGK step (ctypes binding of lbm_oracle.c).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the CPU baseline
leg of the benchmark import this package. The HIP product path never does.

Every function here marshals numpy arrays into the C library; the arithmetic
lives in ``lbm_oracle.c`` and follows Mawson & Revell, Section 3 (Eqs. (2)-(7))
and Section 4.2 (Algorithm 3, the pull iteration).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c99", "-Wall", "-Wextra"]

Q = 19


def build(force: bool = True) -> str:
    """Compile lbm_oracle.c into liblbm_oracle.so next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.orc_tables.argtypes = [ip, dp, ip]
        L.orc_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.orc_collide_cell.argtypes = [dp, dp, ctypes.c_double, dp]
        L.orc_collide_jacobian.argtypes = [dp, dp, ctypes.c_double, dp, dp, dp]
        L.orc_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, ctypes.c_double, dp,
                               dp, dp, ctypes.c_int, dp, dp]
        L.orc_step.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, ctypes.c_double, dp,
                              dp, dp, ctypes.c_int, ctypes.c_int, dp]
        L.orc_run.restype = ctypes.c_int
        L.orc_macros.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, dp, dp, dp, dp, dp]
        L.orc_init_equilibrium.argtypes = [ctypes.c_size_t, dp, dp, dp]
        L.orc_round_half.argtypes = [ctypes.c_double]
        L.orc_round_half.restype = ctypes.c_double
        L.orc_round_bf16.argtypes = [ctypes.c_double]
        L.orc_round_bf16.restype = ctypes.c_double
        L.orc_quantize.argtypes = [ctypes.c_size_t, ctypes.c_int, dp, dp]
        L.orc_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, ctypes.c_double,
                                  dp, dp, dp, ctypes.c_int, dp, dp, dp]
        L.orc_adjoint.restype = ctypes.c_int
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _flags(flags, N):
    if flags is None:
        return None, None
    f = np.ascontiguousarray(flags, dtype=np.uint8).reshape(N)
    return f, f.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def tables():
    """(E [19,3] int, W [19] float64, OPP [19] int) as the oracle holds them."""
    e = (ctypes.c_int * (Q * 3))()
    w = (ctypes.c_double * Q)()
    o = (ctypes.c_int * Q)()
    lib().orc_tables(e, w, o)
    return (np.array(e[:], dtype=np.int64).reshape(Q, 3), np.array(w[:]),
            np.array(o[:], dtype=np.int64))


def equilibrium(rho, u):
    u = _f64(u, (3,))
    out = np.empty(Q)
    lib().orc_equilibrium(float(rho), _dp(u), _dp(out))
    return out


def collide_cell(p, F, tau):
    p = _f64(p, (Q,))
    F = _f64(F if F is not None else np.zeros(3), (3,))
    out = np.empty(Q)
    lib().orc_collide_cell(_dp(p), _dp(F), float(tau), _dp(out))
    return out


def collide_jacobian(p, F, tau):
    """(J [19,19] = ds/dp, dF [19,3] = ds/dF, dtau [19] = ds/dtau)."""
    p = _f64(p, (Q,))
    F = _f64(F if F is not None else np.zeros(3), (3,))
    J = np.empty(Q * Q)
    dF = np.empty(Q * 3)
    dt = np.empty(Q)
    lib().orc_collide_jacobian(_dp(p), _dp(F), float(tau), _dp(J), _dp(dF), _dp(dt))
    return J.reshape(Q, Q), dF.reshape(Q, 3), dt


def init_equilibrium(N, rho=None, u=None):
    """f [19, N] = f^eq(rho, u); rho [N] or None (=1), u [3, N] or None (=0)."""
    rho = _f64(rho, (N,)) if rho is not None else None
    u = _f64(u, (3 * N,)) if u is not None else None
    f = np.empty((Q, N))
    lib().orc_init_equilibrium(N, _dp(rho), _dp(u), _dp(f))
    return f


class Lattice:
    """Box geometry and parameters for the oracle's step functions."""

    def __init__(self, nx, ny, nz, tau, flags=None, uw=(0.0, 0.0, 0.0), force=None,
                 force_field=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.N = self.nx * self.ny * self.nz
        self.tau = float(tau)
        self.flags, self._flags_p = _flags(flags, self.N)
        self.uw = _f64(uw, (3,))
        self.force = _f64(force, (3,)) if force is not None else None
        self.force_field = _f64(force_field, (3 * self.N,)) if force_field is not None else None

    def step(self, s, collide=True):
        s = _f64(s, (Q, self.N))
        out = np.empty_like(s)
        rc = lib().orc_step(self.nx, self.ny, self.nz, self._flags_p, self.tau, _dp(self.uw),
                            _dp(self.force_field), _dp(self.force), int(bool(collide)), _dp(s),
                            _dp(out))
        if rc != 0:
            raise ValueError(f"orc_step failed ({rc}: -1 bad flag value, -3 unsolvable on-site node)")
        return out

    def run(self, s, nsteps, collide=True):
        s = np.array(_f64(s, (Q, self.N)), copy=True)
        rc = lib().orc_run(self.nx, self.ny, self.nz, self._flags_p, self.tau, _dp(self.uw),
                           _dp(self.force_field), _dp(self.force), int(bool(collide)),
                           int(nsteps), _dp(s))
        if rc != 0:
            raise ValueError(f"orc_run failed ({rc}: -1 bad flag value, -2 out of memory, "
                             "-3 unsolvable on-site node)")
        return s

    def macros(self, s):
        s = _f64(s, (Q, self.N))
        rho = np.empty(self.N)
        u = np.empty((3, self.N))
        lib().orc_macros(self.nx, self.ny, self.nz, self._flags_p, _dp(self.force_field),
                         _dp(self.force), _dp(s), _dp(rho), _dp(u))
        return rho, u

    def adjoint(self, s0, T, g):
        """(grad_F [3, N], grad_tau) of L(u(T)) given g = dL/du(T) [3, N]."""
        s0 = _f64(s0, (Q, self.N))
        g = _f64(g, (3 * self.N,))
        ff = self.force_field
        if ff is None and self.force is not None:
            ff = np.ascontiguousarray(np.repeat(self.force[:, None], self.N, axis=1).reshape(-1))
        gF = np.empty(3 * self.N)
        gt = ctypes.c_double(0.0)
        rc = lib().orc_adjoint(self.nx, self.ny, self.nz, self._flags_p, self.tau, _dp(self.uw),
                               _dp(ff), _dp(s0), int(T), _dp(g), _dp(gF), ctypes.byref(gt))
        if rc == -1:
            raise ValueError("the oracle adjoint does not cover on-site velocity nodes")
        if rc != 0:
            raise MemoryError("orc_adjoint could not allocate its state history")
        return gF.reshape(3, self.N), gt.value


def round_half(v: float) -> float:
    return lib().orc_round_half(float(v))


def round_bf16(v: float) -> float:
    return lib().orc_round_bf16(float(v))


def quantize(f, fmt):
    """w_i + round(f_i - w_i) in 'f16' or 'bf16', or float32 of f ('f32')."""
    code = {"f32": 0, "f16": 1, "bf16": 2}[fmt]
    f = _f64(f)
    out = np.empty_like(f)
    lib().orc_quantize(f.size // Q, code, _dp(f), _dp(out))
    return out


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of later oracle calls (OpenMP builds only)."""
    lib().orc_set_num_threads(int(n))
