"""FP64 CPU oracle of the MPBP objective and gradient (test infrastructure only)."""
from . import mpbp_oracle  # noqa: F401
