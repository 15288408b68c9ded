"""MI355X (gfx950) implementation of the P-SWA wavefront context model.

The compute path is the HIP library libpswa.so (C ABI in include/pswa.h);
`pswa` is its thin ctypes binding. Importing the package fails loudly when
the library is not built: there is no CPU fallback.
"""
from . import pswa  # noqa: F401
from .pswa import (  # noqa: F401
    Model, PswaError, decode_frame, pswa_cdf_select, pswa_cdf_tables, pswa_decode_begin,
    pswa_decode_end, pswa_decode_step, pswa_encode_params, pswa_num_steps, pswa_range_decode_seq,
    pswa_range_encode, pswa_range_encode_seq, pswa_state_bytes,
)
