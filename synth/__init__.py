"""Seeded synthetic inputs: reaction mechanisms and thermochemical states.

This package only draws inputs.  It evaluates none of the rate, equilibrium,
thermodynamic or transport formulas that the library and the oracle compute;
both sides read the mechanism text and the arrays it produces.
"""
from .mech import (MechSpec, MECH_C0, MECH_C1, MECH_C4, generate_mechanism, write_mechanism, mechanism_text,
                   with_rate_shift, MECH_V, generate_variant_mechanism)
from .state import (state_c0, state_c1, state_c3_cotangent, state_c4_launch, state_c4_launch_device, c4_element_counts,
                    c1_anchor_requests, load_anchors, gll_nodes,
                    dirichlet_rows)

__all__ = [
    "state_c4_launch_device",
    "with_rate_shift", "MECH_V", "generate_variant_mechanism",
    "MechSpec", "MECH_C0", "MECH_C1", "MECH_C4", "generate_mechanism", "write_mechanism",
    "mechanism_text", "state_c0", "state_c1", "state_c3_cotangent", "state_c4_launch",
    "c4_element_counts", "dirichlet_rows",
]
