"""EBIC population evaluation on MI355X (gfx950).

``Context`` holds a matrix on one GPU; ``Context.evaluate`` and
``Context.evaluate_device`` score a CBF population (row counts, Eq. (1)
fitness and optionally row masks) with the HIP kernels of ``libebic.so``.
``evolve`` runs EBIC on a context, ``Batch`` evaluates or evolves many
matrices together, ``Mlp`` and ``evolve_surrogate`` provide the surrogate
screen, ``mask_rows`` and ``match_scores`` give Step 6's row lists and the
recovery / relevance scores on the device.

The names below are loaded from the compiled library on first use (so that
``python -m paper_1801_03039_amd.build`` works whatever is built); there is no
CPU fallback: using them without a built library raises ``ImportError``.
"""
_EXPORTS = (
    "Batch", "Context", "EbicError", "EBIC_PATH_AUTO", "EBIC_PATH_DIRECT", "EBIC_PATH_INDEX",
    "LIB_PATH", "EvolveConfig", "EvolveResult", "Generation", "Mlp", "Run", "Trend", "evolve",
    "evolve_surrogate", "evolve_screened_with", "evolve_oversampled", "evolve_with", "make_params", "mask_words", "mask_rows",
    "match_scores", "binding",
)

__all__ = list(_EXPORTS)


def __getattr__(name):
    if name in _EXPORTS:
        import importlib
        binding = importlib.import_module(__name__ + ".binding")
        return binding if name == "binding" else getattr(binding, name)
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
