"""MI355X-native hot path of iterative hard thresholding (IHT) for GWAS model selection.

The compute path lives in the HIP/C-ABI library ``libiht.so`` (see ``include/iht.h``); the
``iht`` module is its ctypes binding. Importing the package loads nothing: ``synth`` (seeded
inputs) stays usable without a GPU or a built library.
"""
__all__ = ["iht", "synth"]
