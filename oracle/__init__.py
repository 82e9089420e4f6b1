"""FP64 CPU oracle (test infrastructure only; see fsei_oracle.py and viscous_oracle.py)."""
from .fsei_oracle import *  # noqa: F401,F403
from .fsei_oracle import Grid, PERIODIC, WALL  # noqa: F401
from . import viscous_oracle as viscous  # noqa: F401
from . import momentum_oracle as momentum  # noqa: F401
from . import ibm_oracle as ibm  # noqa: F401
