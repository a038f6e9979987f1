"""FP64 CPU oracle (test infrastructure only; never called by the product path)."""
from .tucker_oracle import *  # noqa: F401,F403
