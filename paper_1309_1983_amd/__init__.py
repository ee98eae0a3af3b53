"""MI355X (gfx950) D3Q19 lattice Boltzmann hot path.

The fused pull stream-collide step of Mawson & Revell (Section 4.2,
Algorithm 3) as hand-written HIP kernels behind the C ABI in include/lbm.h,
with 16-bit offset storage, an in-place AA pattern and a checkpointed
discrete adjoint. This package is the thin Python binding: `Lattice`
(one lattice in device memory), `rollout` (autograd over the adjoint) and the
build step.
"""
from ._abi import LBMError, lib, lib_path  # noqa: F401
from .lattice import Lattice, copy_f32  # noqa: F401
from .autograd import rollout  # noqa: F401

__all__ = ["Lattice", "rollout", "copy_f32", "LBMError", "lib", "lib_path"]
