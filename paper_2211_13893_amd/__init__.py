"""MI355X-native local spectral stage of MS-GFEM with A-harmonic local spaces.

Importing the package loads nothing native; ``paper_2211_13893_amd.msgfem``
is the binding of the HIP library (``libmsgfem.so``) and
``paper_2211_13893_amd.synth`` the seeded input generator.
"""
__all__ = ["synth", "msgfem"]
