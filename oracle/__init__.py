"""FP64 CPU oracle (TEST INFRASTRUCTURE ONLY -- never imported by the product path)."""
from . import ht_oracle, brute  # noqa: F401
