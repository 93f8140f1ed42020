"""MI355X library for the multiphase lattice Boltzmann model with self-tuning
equation of state (Huang, Wu & Adams, arXiv:1809.02390).

The compute path is the HIP library ``liblbm.so`` (C ABI in ``include/lbm.h``);
``paper_1809_02390_amd.lbm`` is its thin ctypes binding.  Importing the
package fails if the library has not been built (``python
paper_1809_02390_amd/build.py``): there is no CPU fallback.
"""
from .lbm import (  # noqa: F401
    LBM_BF16, LBM_FP16, LBM_FP32, Lattice, LbmError, lbm_adjoint_bytes, lbm_adjoint_get, lbm_adjoint_init,
    lbm_adjoint_run, lbm_adjoint_seed, lbm_adjoint_step, lbm_adjoint_theta, lbm_checkpoint_bytes, lbm_create,
    lbm_derive, lbm_derived, lbm_destroy, lbm_get_derived, lbm_get_state, lbm_init, lbm_last_error,
    lbm_load_state, lbm_moments, lbm_param_jacobian, lbm_params, lbm_ref_bytes, lbm_save_state, lbm_set_state,
    lbm_set_stream, lbm_sigma_paper, lbm_state_bytes, lbm_step, lbm_step_saved, lbm_step_saved_chain, lbm_time,
    make_params,
)
from .rollout import LBMRollout, Rollout, choose_every, lbm_rollout  # noqa: F401
