"""FP64 CPU oracle (test infrastructure only; see kde_oracle, lscv_oracle and mlp_oracle)."""
from .kde_oracle import *  # noqa: F401,F403
from .kde_oracle import TAU_DEFAULT  # noqa: F401
from .lscv_oracle import (  # noqa: F401
    binned_pair_sum, chol_params, from_chol_params, lscv_binned, lscv_binned_terms, lscv_direct, nelder_mead,
    pair_sum,
)
from . import mlp_oracle  # noqa: F401,E402
