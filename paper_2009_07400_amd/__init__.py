"""MI355X (gfx950) implementation of tinyMD's Lennard-Jones MD hot path.

The work runs in hand-written HIP kernels behind the C ABI of include/tmd.h
(libtinymd_amd.so, built in-tree by ``build.py``).  ``_abi`` holds the ctypes
binding with the C entry points' names; ``System`` is a thin front end that
uses PyTorch for device memory and streams.  Importing this package does not
need a GPU; using a ``System`` does, and fails loudly without one or without
the built library.
"""

from . import _abi  # noqa: F401
from ._abi import TmdError, TmdParams, load_library  # noqa: F401
from .autograd import LJMDFunction, lj_md  # noqa: F401
from .system import System, compute_forces_static, make_params  # noqa: F401

__all__ = ["System", "compute_forces_static", "make_params", "TmdError", "TmdParams", "load_library", "LJMDFunction", "lj_md"]
