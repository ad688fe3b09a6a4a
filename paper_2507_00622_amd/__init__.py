"""MI355X-native ensemble integrator of Hamiltonian systems with chaos
indicators (arXiv 2507.00622): HIP kernels behind the C ABI of
include/chx.h, bound here by ctypes (see chx.py)."""
from . import chx  # noqa: F401
from .chx import (System, Ensemble, ChxError, henon_heiles, fput, quartic, harmonic, double_pendulum, custom, custom_general,  # noqa: F401
                  integrate_ensemble, integrate_ensemble_noalloc, integrate_batched, sali, gali, lyap_spectrum, ld, ld_indicators, grid_hh_section,
                  hh_section_points, ic_fput_modes, ic_quartic, Gate, gate_features, shutdown)
