"""MI355X (gfx950) PDLP: the PDHG hot path of Applegate et al. in hand-written HIP.

The solver lives in libpdlp_hip.so (C ABI in include/pdlp.h); `pdlp` is its binding.
"""
from .pdlp import (OPTIMAL, ITERATION_LIMIT, NUMERICAL_ERROR, NOT_SOLVED, Solver, Batch,  # noqa: F401
                   default_options, lib, schedule, panel_layout, set_host_threads, PdlpError, STATUS_NAMES,
                   ERR_INVALID_ARGUMENT, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_INVALID_STATE)
