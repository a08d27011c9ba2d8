"""CPU FP64 oracle for the AT compressible Navier-Stokes step (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU leg import this package.  The
product library never loads it.  See atns_oracle.h for what it computes and where in the paper
each part comes from.
"""
from .oracle import Oracle, OracleConfig, build, library_path  # noqa: F401
