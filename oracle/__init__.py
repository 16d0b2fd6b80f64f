"""FP64 CPU oracle for the infinite-domain Poisson method (Anderson, arXiv 2108.11871).

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or calls anything in this package; only the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
use it.  It shares no code, tables or constants with the GPU path.

Modules
-------
poisson       the method, step by step, in plain numpy FP64 (dense sine
              matrices, direct stencils, direct boundary quadrature)
closed_forms  exact potentials of the compact radial test densities
screening     boundary values from the screening charge d phi*/dn and a
              corrected surface trapezoidal rule (James-type methods)
quad.c        direct boundary quadrature in plain C (OpenMP over targets)
"""
from . import poisson, closed_forms, screening  # noqa: F401
