"""Plain FP64 CPU oracle (test infrastructure only; see h2ulv_ref)."""
from .h2ulv_ref import *  # noqa: F401,F403
