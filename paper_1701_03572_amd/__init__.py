"""MI355X-native video stabilization hot path (arXiv 1701.03572, Lim et al.).

Importing the package is cheap; the HIP library is loaded by ``paper_1701_03572_amd.vstab``.
"""
__all__ = ["synth"]
