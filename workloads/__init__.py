"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package generates baryon fields and names the workload presets. It holds
none of the transport method's arithmetic: no physics scalars, no random draws
of the method, no allocation, no walk. Both the HIP path and the oracle receive
the arrays made here and nothing else from this package.
"""
from .fields import lognormal_white, grf_k2, uniform_box, sinusoidal_flow, sinusoidal_profile
from .configs import (CosmoParams, BoxSpec, CONFIGS, make_box, batch_specs, escape_slab,
                      DEFAULT_CELL_CM, KPC_CM)

__all__ = ["lognormal_white", "grf_k2", "uniform_box", "sinusoidal_flow", "sinusoidal_profile",
           "CosmoParams", "BoxSpec", "CONFIGS", "make_box", "batch_specs", "escape_slab",
           "DEFAULT_CELL_CM", "KPC_CM"]
