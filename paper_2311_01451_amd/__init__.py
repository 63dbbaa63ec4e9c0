"""MI355X-native randomized strong recursive skeletonization (RSRS).

Importing the package loads nothing native; ``paper_2311_01451_amd.rsrs``
loads ``librsrs.so`` (HIP, gfx950) on first use and raises if it is missing.
``paper_2311_01451_amd.inputs`` holds the seeded synthetic-input generators.
"""
__all__ = ["inputs", "rsrs"]
