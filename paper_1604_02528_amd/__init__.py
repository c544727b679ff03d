"""MI355X-native supernodal selected inversion (arXiv:1604.02528).

The numeric path lives in the shared library built from csrc/ (C ABI in
include/selinv.h): a host symbolic analysis and LDL^T factorization, and HIP
kernels for gfx950 for the normalization, the root-to-leaves selected
inversion and its adjoint.  Importing this package loads that library and
fails loudly if it has not been built.
"""

from .capi import load as _load
from .selinv import SelInv  # noqa: F401
from .autograd import SelInvFunction  # noqa: F401

_load()

__all__ = ["SelInv", "SelInvFunction"]
