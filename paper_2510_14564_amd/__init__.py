"""MI355X-native differentiable tile splatting (3D Gaussian Splatting hot path).

Importing the package does not load the HIP library; ``paper_2510_14564_amd.gs``
does, and fails loudly when it is missing.
"""
__all__ = ["scenes"]
