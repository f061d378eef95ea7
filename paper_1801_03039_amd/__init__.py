"""EBIC population evaluation on MI355X (gfx950).

``Context`` holds a matrix on one GPU; ``Context.evaluate`` and
``Context.evaluate_device`` score a CBF population (row counts, Eq. (1)
fitness and optionally row masks) with the HIP kernels of ``libebic.so``.
The library must be built (``python -m paper_1801_03039_amd.build``); there is
no CPU fallback.
"""
from .binding import (  # noqa: F401
    Batch,
    Context,
    EbicError,
    EBIC_PATH_AUTO,
    EBIC_PATH_DIRECT,
    EBIC_PATH_INDEX,
    LIB_PATH,
    EvolveConfig,
    EvolveResult,
    Generation,
    Mlp,
    Trend,
    evolve,
    evolve_surrogate,
    evolve_with,
    make_params,
    mask_words,
)
