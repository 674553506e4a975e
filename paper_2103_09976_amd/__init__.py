"""MI355X two-site DMRG middle-site library (H_eff psi, blocking, transformation, Davidson).

The compute lives in libdmrg_hip.so (HIP, gfx950) behind the C ABI of
include/dmrg.h; ``paper_2103_09976_amd.dmrg`` is its ctypes binding.
"""
from . import dmrg  # noqa: F401
from .dmrg import (DMRG_LEFT, DMRG_RIGHT, DMRG_SCHEME_CN, DMRG_SCHEME_NC, DMRG_PREC_F32,  # noqa: F401
                   DMRG_PREC_F64, Context, DmrgError, Heff, Isometry, OpSet, load, middle_step)
