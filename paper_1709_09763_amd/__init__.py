"""MI355X (gfx950) implementation of the hot path of Multilevel Sequential^2
Monte Carlo (Latz, Papaioannou, Ullmann, J. Comp. Phys.).

The compute lives in the HIP library ``libmls2mc.so`` (C ABI declared in
``include/mls2mc.h``).  This package is a thin ctypes binding with the same
names: it checks tensor shapes and dtypes, passes device pointers and the
current HIP stream, and raises on a non-zero status.  PyTorch provides device
memory and streams only.
"""
from ._lib import (  # noqa: F401
    FIELD_KAPPA_F32, FIELD_KAPPA_F64, FIELD_LOG_F64, FP64, MIXED, Context, Mls2mcError,
    Problem, RunConfig, lib, library_path, mls2mc_create, mls2mc_destroy, mls2mc_forward,
    mls2mc_forward_field, mls2mc_gather, mls2mc_kl_field, mls2mc_last_error, mls2mc_loglik,
    mls2mc_n_elem, mls2mc_n_obs, mls2mc_n_unknowns, mls2mc_next_step, mls2mc_pcn_step,
    mls2mc_philox_fill, mls2mc_profile, mls2mc_profile_read, mls2mc_resample, mls2mc_run,
    mls2mc_version, PROF_GEMM, PROF_SOLVE, mls2mc_autotune, mls2mc_get_launch, mls2mc_set_launch,
    mls2mc_pcn_step_da, mls2mc_surrogate_add_pairs, mls2mc_surrogate_get_params, mls2mc_surrogate_init,
    mls2mc_surrogate_loss_grad, mls2mc_surrogate_n_pairs, mls2mc_surrogate_n_params,
    mls2mc_surrogate_predict, mls2mc_surrogate_set_params, mls2mc_surrogate_train,
    mls2mc_forward_batch, mls2mc_run_batch, mls2mc_kl_eigenvalues, KERNEL_PCN, KERNEL_RWM,
    SCHEME_MLB, SCHEME_MLS2MC, COV_MATERN32, COV_SEPEXP, BC_DIRICHLET, BC_FLOW_CELL,
    mls2mc_ctx_n_unknowns, mls2mc_decide, DECIDE_ITU, DECIDE_LU, DECIDE_DONE, DECIDE_NEED_CV,
    mls2mc_cv_lu, mls2mc_set_linear_model, mls2mc_set_linear_surrogate, mls2mc_resample_noalloc,
)
