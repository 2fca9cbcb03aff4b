"""MI355X-native catalog shift-and-stack voting transform (arXiv 2509.26279).

The search itself lives in the HIP library ``libsas.so`` (C ABI:
``include/sas.h``); ``sas`` is its Python binding and ``synth`` makes seeded
synthetic catalogs.  Importing the package loads nothing; ``sas.load()``
loads the library and fails loudly when it is not built.
"""
__all__ = ["sas", "synth", "build"]
