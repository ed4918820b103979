"""CPU oracle (test infrastructure only; never used by the product path)."""
from .kspace import Oracle, wavenumbers, alpha_db_to_neper, pml_profile, staggered_mean  # noqa: F401
