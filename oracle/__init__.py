"""FP64 CPU oracle for efunc -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The HIP library never calls it
and shares no code with it.  The C sources (``efunc_oracle.c``) hold the
arithmetic; this module only marshals numpy arrays through ctypes.
``oracle.variants`` (``efunc_oracle_var.c``) covers the model variants:
polynomial degree 0/1/2, key sets and fixed or learnable scales.
"""
from .oracle import (  # noqa: F401
    Grid,
    build_oracle,
    load,
    num_keys,
    threads,
    lattice,
    build_keys,
    eval_global,
    eval_qgrad,
    eval_qgrad_scales,
    eval_cond,
    eval_trunc,
    grad_global,
    grad_trunc,
    grad_theta,
    adam,
    meanshift,
    fit_step,
    NCH,
)
