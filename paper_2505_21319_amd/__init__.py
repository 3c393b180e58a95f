"""MI355X-native engine for the efunc representation (arXiv 2505.21319).

The compute path is the C-ABI library libefunc.so (HIP kernels for gfx950);
`efunc` is its Python binding.
"""
from .efunc import (  # noqa: F401
    EXPORTS,
    Engine,
    EfuncError,
    efunc_create,
    efunc_default_adam,
    efunc_default_config,
    efunc_destroy,
    efunc_eval,
    efunc_fit_step,
    efunc_get_stats,
    efunc_grad,
    efunc_init_params,
    efunc_read_timing,
    efunc_set_timing,
    lib,
)
