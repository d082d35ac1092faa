"""FP64 CPU oracle (test infrastructure only; see tsvd_oracle's header)."""
from .tsvd_oracle import *  # noqa: F401,F403
