"""MI355X (gfx950) amplitudes of random quantum circuits by sliced tensor-network contraction.

The compute path is libqflex.so (HIP kernels behind the C ABI in include/qflex.h); this
package only marshals arguments to it.  Nothing here falls back to a CPU implementation.
"""
from .qflex import (Grid, build_grid, fidelity_samples, frugal_sample,  # noqa: F401
                    plan_describe, select_slices, with_fsim_angles)
try:
    from .qflex import Amplitudes  # noqa: F401
except ImportError:  # pragma: no cover
    pass
