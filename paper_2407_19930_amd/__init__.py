"""MI355X (gfx950) library for the space-time chi0 -> RPA correlation-energy path
(LRI / NAO low-scaling RPA, arXiv 2407.19930): hand-written HIP kernels behind a
C ABI (include/rpa_mi355x.h) and a thin ctypes binding (binding.py)."""
from .binding import (Batch, Context, Plan, RpaError, Session, Tuning, build_chi0_tau, build_green_tau,  # noqa: F401
                      chi0_R_to_q, chi0_tau_to_omega, load, rpa_check_green_symmetry, rpa_correlation_energy,
                      rpa_correlation_energy_noalloc, rpa_ec_workspace_size, rpa_green_workspace_size,
                      rpa_noalloc_scratch_bytes)
