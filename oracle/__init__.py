"""FP64 CPU oracle of the seismic saliency method (Shafiq et al., ICIP 2017).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of the
benchmark are the only users.  Nothing here is shared with the GPU path.
"""
from .oracle import *  # noqa: F401,F403
