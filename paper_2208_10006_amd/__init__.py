"""MI355X-native SBR (shooting-and-bouncing-ray) channel simulator.

Importing the package loads nothing native; ``paper_2208_10006_amd.sbr``
loads the HIP library (``libsbr.so``) and fails loudly when it is missing.
"""
__all__ = ["workloads"]
