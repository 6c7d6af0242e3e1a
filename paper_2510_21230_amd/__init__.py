"""atm3: linked-cell Lennard-Jones + Axilrod-Teller-Muto forces on MI355X.

Hand-written HIP kernels for gfx950 behind the C ABI of ``libatm3.so``
(``include/atm3.h``); this package only marshals torch device tensors into
that ABI.  ``Mlp`` is the learned three-body pair surrogate (descriptors,
BF16 MFMA pair MLP, training, exact fallback).  ``workloads`` draws the
seeded synthetic inputs; ``md_run`` is the velocity-Verlet driver and ``md_nvt``
its constant-temperature form.
"""
from ._lib import (MLP_NPARAM, Atm3Error, Context, Mlp, TERM_ATM, TERM_LJ, bin_cells,  # noqa: F401
                   compute_forces, context, load, make_params, md_nvt, md_run)

__all__ = ["Atm3Error", "Context", "MLP_NPARAM", "Mlp", "TERM_ATM", "TERM_LJ", "bin_cells", "compute_forces",
           "context", "load", "make_params", "md_nvt", "md_run"]
