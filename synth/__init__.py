"""Seeded synthetic inputs shared by the oracle and the GPU path (no method
arithmetic lives here)."""
from .workloads import (ALL_OPS, BINARY_OPS, UNARY_OPS, STANDARD_OPS,
                        WORKLOADS, make, tiny, units16, multitarget16,
                        batch128, large24, random_small, subspace3000, subspace512)
