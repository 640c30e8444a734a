"""CPU FP64 oracle for the fast cascade (Beylkin, "Fast convolution algorithm for
state space models", arXiv 2411.17729).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it. It shares no code with the HIP
library (no kernels, headers, helpers or constant tables) and it never imports
``paper_2411_17729_amd``.
"""

from .ssm_oracle import (  # noqa: F401
    trapezoid,
    trapezoid_adjoint,
    zoh,
    zoh_adjoint,
    recursion,
    powers,
    impulse_response,
    truncated_sum,
    truncated_sum_fft,
    cascade,
    transfer,
    transfer_truncated,
    grads_recursion,
    grads_truncated_bruteforce,
    grads_full,
    effective_stages,
    auto_stages,
    free_response,
)
from .ssm_plr import (  # noqa: F401
    plr_compress,
    plr_dense,
    plr_apply,
    plr_ranks,
    plr_flops,
    plr_error_bound,
    cascade_plr,
)
