"""ta: execution-trace -> rank x iteration x region tensor analysis on MI355X.

Importing the package loads nothing native; ``paper_2605_03561_amd.ta`` binds
the HIP library (and fails loudly if it has not been built), and
``paper_2605_03561_amd.synth`` is the seeded input generator.
"""
__all__ = ["ta", "synth"]
