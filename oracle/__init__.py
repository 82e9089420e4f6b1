"""FP64 CPU oracle (test infrastructure only; see fsei_oracle.py)."""
from .fsei_oracle import *  # noqa: F401,F403
from .fsei_oracle import Grid, PERIODIC, WALL  # noqa: F401
