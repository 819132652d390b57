"""MI355X (gfx950) coherent-dedispersion correlator.

The path runs in the HIP library libddx.so (C ABI in include/ddx.h); this
package holds its sources (csrc/), the in-tree build step (build.py) and a thin
ctypes binding (binding.py).  There is no CPU fallback: without the built
library every call raises.
"""
from .binding import (  # noqa: F401
    Plan, plan_blocking, layout_blockings, Cnn, Chirp, ChirpBank, Image, incoherent_delays, power_beam, incoherent_dedisperse, tree_dedisperse,
    tree_dedisperse_static, TREE_STATIC_MAX,
    chimg_preintegrate, chimg_trajectories, chimg_gradient_sums, chimg_cells, chimg_preintegrate_cells,
    chimg_sampling_blocks, chimg_trajectories_ext, chimg_cells_2d, chimg_preintegrate_2d, chimg_trajectories_2d,
    DdxError, lib, LIB_PATH, SIGNATURES,
    OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ESIZE, EFULL, EUNSUPPORTED,
    IN_CI8, IN_CF32, CORR_F32, CORR_F16, CORR_E4M3, OUT_PACKED, OUT_FULL, FLUSH,
)
