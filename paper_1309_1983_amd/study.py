"""Binding of the memory-access study kernels (include/lbm_study.h).

Marshals torch device tensors into the study entry points; every kernel runs
in the HIP library. The study re-measures on gfx950 the access-pattern
experiments of Mawson & Revell, Section 4.3.
"""
from __future__ import annotations

import ctypes

import torch

from . import _abi

STREAM_MODES = {"copy": 0, "read": 1, "write": 2}
SHIFT_METHODS = {"direct": 0, "lds": 1, "dpp": 2, "direct4": 3}
SCHEMES = {"pull": 0, "push": 1}


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def stream(mode, src, dst, sink, n, nvec, roff=0, woff=0, width=4, stream=None):
    _abi.check(_abi.lib().lbm_study_stream(STREAM_MODES[mode], _p(src), _p(dst), _p(sink),
                                           ctypes.c_size_t(n), nvec, roff, woff, width, _s(stream)),
               "lbm_study_stream")


def shift(src, dst, nx, nrows, method, stream=None):
    _abi.check(_abi.lib().lbm_study_shift(_p(src), _p(dst), nx, nrows, SHIFT_METHODS[method],
                                          _s(stream)), "lbm_study_shift")


def planes(mode, src, dst, sink, nx, ny, nz, stream=None):
    _abi.check(_abi.lib().lbm_study_planes(STREAM_MODES[mode], _p(src), _p(dst), _p(sink), nx, ny, nz,
                                           _s(stream)), "lbm_study_planes")


def step(a, b, flags, nx, ny, nz, tau, scheme, block_x=256, stream=None):
    _abi.check(_abi.lib().lbm_study_step(_p(a), _p(b), _p(flags), nx, ny, nz, ctypes.c_float(tau),
                                         SCHEMES[scheme], block_x, _s(stream)), "lbm_study_step")
