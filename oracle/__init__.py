"""Exact CPU oracle for the reproducible PBiCGStab hot path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the GPU library.  It shares no
code with the GPU library.  The arithmetic lives in ``rpk_oracle.c`` (a big-
integer exact accumulator and the two solver loops); this module only builds
and loads that shared object and marshals numpy arrays.
"""
from .oracle import (build, load, exdot, exspmv, jacobi, solve, set_threads,
                     get_threads, HIST_W, STATUS, STD, PIPELINED)

__all__ = ["build", "load", "exdot", "exspmv", "jacobi", "solve", "set_threads",
           "get_threads", "HIST_W", "STATUS", "STD", "PIPELINED"]
