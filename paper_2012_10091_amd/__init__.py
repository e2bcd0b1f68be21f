"""MI355X (gfx950) multigrid ensemble Kalman filter hot path.

The computation lives in libmenkf.so (HIP kernels behind the C ABI of
include/menkf.h); this package only loads it and marshals torch tensors.
"""

from .binding import (  # noqa: F401
    Batch, Context, Graph, MenkfError, Net, Trainer, pack_params, unpack_params, config_from, make_config, ram_ratio, last_error,
    MENKF_BURGERS1D, MENKF_NS2D, MENKF_BURGERS1D_INLET, MENKF_EULER1D_INLET, MENKF_F32, MENKF_F64, MENKF_GAIN_EXACT_R, MENKF_GAIN_SAMPLE_EE, MENKF_GAIN_ENSEMBLE_SPACE,
    MENKF_FINE, MENKF_COARSE, MENKF_PROLONG_PLAIN, MENKF_PROLONG_LEARNED, MENKF_PROLONG_LEARNED_FALLBACK,
    MENKF_CYCLE_DEVICE,
)
from ._lib import load as load_library, LIB_PATH  # noqa: F401
