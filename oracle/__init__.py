"""FP64 CPU oracle for the sloshing step and the wrench surrogate.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the product path never does.  It
shares no code with the HIP path.

* ``oracle.sph`` -- ctypes binding of ``sph_oracle.c`` (FP64, plain C).
* ``oracle.mlp`` -- the surrogate network in NumPy float64.
"""
