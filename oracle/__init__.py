"""Float64 CPU oracle for primed PCA.  Test infrastructure only: imported by
tests/, the smoke check and the benchmark's CPU-baseline leg, never by the
GPU library or its Python binding."""
from .ppca_oracle import *  # noqa: F401,F403
