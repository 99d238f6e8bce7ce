"""FP64 CPU oracle of the NLPR fusion ADMM (test infrastructure only; see nlpr_oracle)."""
from .nlpr_oracle import *  # noqa: F401,F403
from . import nlpr_oracle  # noqa: F401
