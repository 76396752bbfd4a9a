"""FP64 CPU oracle for HOQRI (test infrastructure; see hoqri_ref)."""
from .hoqri_ref import *  # noqa: F401,F403
