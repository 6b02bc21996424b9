"""MI355X-native domain-wall Dirac operator and Krylov solver (qdwf).

The product is the C-ABI library ``libqdwf.so`` (declared in ``include/qdwf.h``)
built from the HIP sources in ``csrc/``. ``paper_2112_01852_amd.qdwf`` is its
thin ctypes binding; ``paper_2112_01852_amd.inputs`` draws seeded synthetic
inputs. Importing this package loads nothing; the binding loads the library on
first use and raises if it is missing.
"""
