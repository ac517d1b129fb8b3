"""FP64 CPU oracle for ACCORD-FBS.  TEST INFRASTRUCTURE ONLY: imported by tests,
the smoke check and the benchmark's CPU-baseline leg; never by the GPU path."""
from .accord_oracle import *  # noqa: F401,F403
from .accord_oracle import (FitResult, brute_column, diag_root, fit_cd, fit_fbs,  # noqa: F401
                            grad, kkt_residual, lipschitz, line_search_test, objective,
                            prox, smooth, soft_threshold)
from .mx_oracle import (E4M3_MAX, MX_BLOCK, e4m3_round, e4m3_value, fit_fbs_mx,  # noqa: F401
                        mx_quantize, mx_scale_exp)
from . import adjoint_oracle  # noqa: F401
from . import tuning_oracle  # noqa: F401
