"""FP64 CPU oracle (test infrastructure only; see mrpie64.py)."""
from .mrpie64 import *  # noqa: F401,F403
from .mrpie64 import __all__  # noqa: F401
