"""MI355X-native MPPI sampling step for reference-free drone racing.

Importing the package loads nothing; ``paper_2509_14726_amd.mppi`` binds the
HIP library (``libmppi.so``) and fails loudly when it is missing.
"""
__all__ = ["mppi", "synth"]
