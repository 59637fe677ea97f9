"""MI355X-native particle-mesh force step and reverse-time adjoint (pmwd method).

The compute path is libpmx.so (hand-written HIP for gfx950 behind the C ABI of
include/pm.h); this package only loads it and marshals arguments.
"""
from ._lib import EXPORTS, N_FILTER_PARAMS, PMError, load  # noqa: F401
from .api import (PMContext, Simulate, config_from_workload, host_tables,  # noqa: F401
                  make_config, simulate, workspace_bytes)
