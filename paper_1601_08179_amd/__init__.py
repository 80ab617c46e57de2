"""MI355X (gfx950) statically condensed spectral-element Helmholtz solver.

The HIP library ``libsemcond.so`` (built by ``paper_1601_08179_amd.build``)
implements the operator, the preconditioner and the solver; ``semcond`` is its
ctypes binding.
"""
