"""MI355X (gfx950) implementation of the data-parallel hot path of primed PCA.

The compute runs in the HIP library libppca.so (see include/ppca.h); this
package is its thin Python binding.  Build with
`python -m paper_2109_03709_amd.build`.
"""
from ._lib import (  # noqa: F401
    BF16, F32, FP8_E4M3, MAX_K, OP_CENTER, OP_EIGENGAME, OP_OJA, OP_POWER, OP_PROJECT, OP_RR, OP_STREAM, OP_POWER_SEQ,
    Data, GROUP_ITEM_CANDIDATES, NOALLOC_SCRATCH_BYTES, GROUP_MAX_D, GROUP_MAX_K, Group, PPCAError, Problem, center_quantize,
    grouped_workspace_bytes, kernel_stats, lib, ppca, prime_eigengame, prime_oja, prime_power,
    prime_power_eps, prime_power_grouped, prime_power_seq, project_gram, project_gram_rows, rayleigh_ritz, read_probe, rayleigh_ritz_grouped, rayleigh_ritz_noalloc, set_chunk_rows, set_fused_pass,
    set_group_item_bytes, set_kernel_timing, stream_pass, strerror, tune_group_items,
    workspace_bytes,
)
