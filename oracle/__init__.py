"""ORACLE -- test infrastructure only.

A plain, slow FP64 CPU implementation of the steady non-gray phonon BTE-RTA
solve (sequential and synthetic iterations, first-order upwind finite volume,
discrete ordinates).  It exists to check the GPU library and shares no code
with it.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it.

Parity status of each function (what pins it) is recorded in the tests under
tests/test_oracle_*.py.
"""
from .solver import (OracleError, Result, Setup, accel_state, accel_unpack, anderson_next,  # noqa: F401
                     boundary_flows, boundary_inflow, diffusion_operator, divergence, energy_defect,
                     equilibrium, fourier_guess, lsq_weights, moments, prepare, reconstruct, reconstruct_fields,
                     solve, solve_system_order2, source, threads, transport, transport_systems)
