"""MI355X (gfx950) optimal multiple sequence alignment by k-dimensional DP.

The compute path is the HIP library ``_lib/libmsa_dp.so`` (C ABI in
``include/msa_dp.h``); this package is its Python binding.  Build with
``python -m paper_2311_17530_amd.build``.
"""
from ._lib import (  # noqa: F401
    GAP,
    MAX_K,
    MSA_COOPTIMAL,
    MSA_EAGAIN,
    MSA_EDEVICE,
    MSA_EINVAL,
    MSA_END_GAPS_FREE,
    MSA_ENOMEM,
    MSA_ERANGE,
    MSA_ESHUTDOWN,
    MSA_OK,
    MSA_NEAROPT,
    MSA_PRUNE,
    DeviceAligner,
    MsaError,
    Server,
    align,
    align_batch,
    align_coopt,
    align_nearopt,
    exported_names,
    lib,
    check_scoring,
    score_bounds,
    strerror,
    tile_edge,
    tile_grid,
    wave_counts,
    workspace_bytes,
    workspace_bytes_ex,
)
