"""MI355X-native per-grid-point thermochemistry (HIP kernels behind a C ABI).

Production rates, heat release, NASA-7 thermodynamics, mixture-averaged
transport, and the vector-Jacobian product and dense Jacobian of the
production rates, in FP64 or mixed FP32/FP64, for the chemistry source terms of
a low-Mach reacting-flow solver (nekCRF, Section 2).
"""
from .api import (CrfError, Mechanism, WdotFn, hbm_budget, new_workspace, reactor_step, reactor_workspace,
                  source, species_major, thermo, transport, wdot, wdot_fwd, wdot_jac, wdot_jvp, wdot_vjp,
                  workspace_bytes)

__all__ = ["CrfError", "Mechanism", "WdotFn", "hbm_budget", "new_workspace", "reactor_step", "reactor_workspace",
           "source", "species_major", "thermo", "transport", "wdot", "wdot_fwd", "wdot_jac", "wdot_jvp", "wdot_vjp",
           "workspace_bytes"]
