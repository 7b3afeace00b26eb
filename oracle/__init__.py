"""FP64 CPU oracle (test infrastructure only; see ``nmg_oracle``)."""
from .nmg_oracle import *  # noqa: F401,F403
