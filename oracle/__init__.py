"""CPU oracle for the phaseless-AFQMC walker step.

Test infrastructure only: used by the tests, the smoke check and the benchmark's
CPU baseline.  The product path never imports it."""
from . import afqmc_oracle  # noqa: F401
