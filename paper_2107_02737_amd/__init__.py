"""MI355X (gfx950) DNN-SP2 density-matrix solver.

The product is the HIP library ``lib/libsp2.so`` behind the C ABI of
``include/sp2.h``; this package only marshals torch tensors into it.  There
is no CPU fallback: importing the API without the built library raises.
"""

from ._lib import (EXPORTED, PRECISIONS, SP2Error, allocate_workspace, load_library,  # noqa: F401
                   make_options, sp2_bounds, sp2_default_options, sp2_density, sp2_density_ex,
                   sp2_jvp, sp2_last_error, sp2_layer, sp2_spectral_bounds, sp2_split, sp2_vjp,
                   sp2_workspace_bytes, sp2_mulliken, sp2_xl_scratch_bytes, allocate_xl_scratch,
                   sp2_xl_response, sp2_xl_kernel, SP2_XL_MAX_RANK, nvt_params,
                   sp2_nvt_gamma_tc, sp2_nvt_first_half, sp2_nvt_second_half, sp2_history,
                   sp2_density_noalloc, sp2_homo_lumo)
from .sp2 import SP2Density, density, homo_lumo, jvp, vjp  # noqa: F401
