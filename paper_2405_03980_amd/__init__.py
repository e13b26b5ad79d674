"""MI355X-native hot path of the two-fluid SPH model with spin angular momentum
(rotating liquid helium-4, explicit weakly-compressible SPH).

The computation lives in the HIP library libsph4he.so (C ABI: include/sph4he.h).  This
package holds its ctypes binding (`_lib`), torch-backed handles (`sim`), the seeded input
generators (`inputs`), the autotuner (`tune`) and the build script (`build`).
"""
from . import inputs  # noqa: F401
from ._lib import FP32_MIXED, FP64, SphError  # noqa: F401


def __getattr__(name):
    if name in ("Simulation", "Batch", "simulation_from", "batch_from"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
