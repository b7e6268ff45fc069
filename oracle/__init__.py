"""FP64 CPU oracle for TT arithmetic (test infrastructure, see tt_oracle)."""
from .tt_oracle import *  # noqa: F401,F403
from .tt_oracle import __all__  # noqa: F401
