"""FP64 CPU oracle (test infrastructure only; never part of the product path)."""
from .cfog_oracle import *  # noqa: F401,F403
