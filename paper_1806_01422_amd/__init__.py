"""MI355X-native matrix-free spectral-element viscous-Burgers operators F(u), J(u)v, J(u)^T w,
RK4 forward/adjoint integration and batched uneven problems (arXiv 1806.01422), backed by the HIP
library libsem (include/sem.h)."""
from .sem import (EXPORTED, LIB_PATH, SCHEMES, Batch, Context, SemError, SEMRhs, SEMTrajectory, lib,  # noqa: F401
                  SEMTrajectoryRevolve, SEMTrajectoryStored, probe_fp64_rates, revolve_plan, trajectory,
                  trajectory_revolve, trajectory_stored)
