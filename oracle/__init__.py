"""FP64 CPU oracle (test infrastructure only; see ``oracle.gs``)."""
from .gs import *  # noqa: F401,F403
