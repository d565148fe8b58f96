"""MI355X (gfx950) matched-filter / projected-gradient MRF reconstruction.

The computation lives in libmrf.so (HIP kernels behind the C ABI of
include/mrf.h); this package holds its sources (csrc/), the build script and
a thin ctypes binding (mrf.py) whose functions carry the C names.
"""
from .mrf import (MRF_E_HIP, MRF_E_INVAL, MRF_E_NOCONV, MRF_E_NOMEM, MRF_E_NUMERIC,  # noqa: F401
                  MRF_E_UNSUPPORTED, Dictionary, MrfError, Net, Operator, lib, mrf_dict_copy_atoms,  # noqa: F401
                  mrf_ipg_solve, mrf_ipg_step, mrf_match, mrf_match_local, mrf_match_noalloc, mrf_net_adam,
                  mrf_net_forward, mrf_net_loss_grad, mrf_net_noisy_batch, mrf_net_train,
                  mrf_op_adjoint, mrf_op_forward, mrf_quantize_rows, mrf_version)
