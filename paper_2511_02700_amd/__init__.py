"""MI355X-native solver for two-asset exponential-Levy option PIDEs (the method
of arXiv 2511.02700): hand-written HIP kernels for gfx950 behind the C ABI of
include/lpide.h, with this thin Python binding on top."""

from .api import (Batch, Plan, PricesFn, PsPlan, discretize_host, levy_black_scholes, levy_from_std,  # noqa: F401
                  levy_nts, make_grid, make_payoff, make_ps_grid, plan_from_workload, ps_discretize_host, solve,
                  std_params_of)
from ._lib import LpideError, lib  # noqa: F401
