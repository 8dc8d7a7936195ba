"""MI355X-native hot path of SkipGS-style 3DGS training.

Importing the package loads nothing native; ``paper_2603_08997_amd.skipgs``
binds the HIP library (``libskipgs.so``) and fails loudly if it is missing.
``paper_2603_08997_amd.scenes`` draws the seeded synthetic inputs.
"""
__all__ = ["scenes", "skipgs"]
