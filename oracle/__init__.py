"""CPU FP64 oracle for one implicit-HDG Newton step (test infrastructure).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import or
run anything in this package. It shares no code with the GPU library; its only
shared input is the seeded workload generator `hdg_inputs`.
"""
from .hdg_oracle import *  # noqa: F401,F403
