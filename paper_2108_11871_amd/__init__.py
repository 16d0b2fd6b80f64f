"""MI355X-native infinite-domain Poisson solver (Anderson, arXiv 2108.11871).

phi = G * rho on a uniform rectangular grid, computed as a spectrally
accurate sine-transform Dirichlet solve plus a 4th/6th-order harmonic
correction whose boundary values come from slice-wise FFT convolutions.
All arithmetic runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/ipoisson.h``; this package only marshals arguments.

The HIP library is loaded on first use of a solver entry point; importing
the package (or ``paper_2108_11871_amd.inputs``) does not touch the GPU.
"""

__all__ = [
    "solve",
    "Plan",
    "Batch",
    "SolveFn",
    "PRECISIONS",
    "library_path",
]


def __getattr__(name):
    if name in __all__:
        from . import api

        return getattr(api, name)
    raise AttributeError(name)
