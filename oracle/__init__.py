"""Plain FP64 CPU oracle for the per-point thermochemistry — TEST INFRASTRUCTURE ONLY.

Nothing in the library imports this package.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark use it, to check the GPU results and to time
a plain CPU implementation beside them.

The paper (Section 2) names the quantities its right-hand-side kernels evaluate at
every grid point — the net production rates of Eq. (1a), the heat-release term of
Eq. (1b), the ideal-gas density of Eq. (1d) and the mixture-averaged diffusivities
of Eq. (2) — and defers their definitions to a mechanism "in Cantera format".  The
oracle therefore writes out the standard textbook (Chemkin/Cantera) definitions,
vectorised over points with numpy, in the order those definitions state them.
Every function works for float64 and complex128 inputs, so that complex-step
differentiation of the forward functions can pin the analytic derivatives; every
branch compares real parts only.

Parity status of each part (what pins it) is listed in the module docstrings.
"""
from .mechfile import OracleMech, read_mechanism
from .thermo import mixture_state, nasa7, thermo_properties
from .kinetics import rates_of_progress, production_rates
from .transport import transport_properties
from .jacobian import jacobian, vjp, jvp, complex_step_jacobian, complex_step_jvp, central_fd_jacobian
from .source import chemistry_source
from .reactor import rhs, source_jacobian, ros2_step
from .equil import equilibrate

__all__ = [
    "OracleMech", "read_mechanism", "mixture_state", "nasa7", "thermo_properties",
    "rates_of_progress", "production_rates", "transport_properties", "jacobian", "vjp", "jvp",
    "complex_step_jacobian", "complex_step_jvp", "central_fd_jacobian", "equilibrate",
    "chemistry_source", "rhs", "source_jacobian", "ros2_step",
]
