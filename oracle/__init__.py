"""FP64 CPU oracle (test infrastructure only; see kde_oracle)."""
from .kde_oracle import *  # noqa: F401,F403
from .kde_oracle import TAU_DEFAULT  # noqa: F401
