"""SpInGP hot path for MI355X: temporal-GP inference in sparse-precision form.

The computation lives in the gfx950 library ``libspingp.so`` behind the C ABI of
``include/spingp.h``; ``spingp`` is its thin Python binding and ``autograd`` wraps the log
marginal likelihood and its hand-written gradient as a torch.autograd.Function;
``optimize`` fits hyperparameters by maximum marginal likelihood.
"""
from .spingp import (  # noqa: F401
    MATERN12,
    MATERN32,
    MATERN52,
    MATERN72,
    PERIODIC,
    QUASIPERIODIC,
    SQEXP,
    Handle,
    SpinGPError,
    load_library,
    spingp_assemble,
    spingp_blocks,
    spingp_create,
    spingp_destroy,
    spingp_factor,
    spingp_get_tile,
    spingp_logml,
    spingp_logml_grad,
    spingp_predict,
    spingp_selinv,
    spingp_set_tile,
    spingp_solve,
    spingp_status,
    spingp_tile_count,
    spingp_tile_shape,
    spingp_tune,
    spingp_workspace_bytes,
)
from .optimize import FitResult, fit, scg  # noqa: F401,E402
