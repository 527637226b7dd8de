"""CPU float64 oracle for the full-order implicit cell step (test infrastructure
only: imported by tests, the smoke check and the benchmark's CPU baseline)."""
from .cellmodel import (FARADAY, GAS_R, Geometry, Model, NewtonFailure,  # noqa: F401
                        newton_step, simulate, ocp, f_pre, cutoff_reached,
                        lte_estimate, simulate_adaptive)
from .pod import gram, pod  # noqa: F401,E402
