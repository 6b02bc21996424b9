"""CPU oracle for the domain-wall Dirac operator and its CG solve.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library. It shares no
code with the HIP path; only the seeded input generators are common to both.

* ``oracle.cpu``       -- ctypes front end of ``dwf_oracle.cpp`` (FP64 loops).
* ``oracle.dense``     -- an independent sparse-matrix construction of the same
                          operators from Kronecker products, for small lattices.
* ``oracle.geometry``  -- checkerboard and neighbour tables by enumeration.
* ``oracle.freefield`` -- unit-link closed forms in momentum space.
* ``oracle.streaming`` -- per-site SU(3) product and triad of the memory probes.
"""
