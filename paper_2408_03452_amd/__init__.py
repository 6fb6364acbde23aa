"""Matrix-free TPFA finite-volume conjugate gradient for AMD MI355X (gfx950).

The solver is the HIP library ``libmffv.so`` (C ABI in ``include/mffv.h``);
``paper_2408_03452_amd.mffv`` is its Python binding. Import the binding
explicitly (``from paper_2408_03452_amd import mffv``): it loads torch and the
library, and fails loudly if the library has not been built.
"""
__all__ = ["mffv", "build"]
