"""atm3: linked-cell Lennard-Jones + Axilrod-Teller-Muto forces on MI355X.

Hand-written HIP kernels for gfx950 behind the C ABI of ``libatm3.so``
(``include/atm3.h``); this package only marshals torch device tensors into
that ABI.  ``workloads`` draws the seeded synthetic inputs.
"""
from ._lib import (Atm3Error, Context, TERM_ATM, TERM_LJ, bin_cells, compute_forces, context,  # noqa: F401
                   load, make_params)

__all__ = ["Atm3Error", "Context", "TERM_ATM", "TERM_LJ", "bin_cells", "compute_forces", "context",
           "load", "make_params"]
