"""MI355X-native per-frame Gaussian-splatting rasterizer (AirGS hot path).

Importing the package loads nothing native; ``paper_2512_20943_amd.gs`` is the
binding of the HIP library and raises if the library is not built.
"""
__all__ = ["scenes", "gs"]
