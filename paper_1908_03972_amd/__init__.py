"""pmgfr: MI355X-native P-multigrid FR/CPR stage solver for locally preconditioned low-Mach flow.

The computation lives in the HIP library ``libpmgfr.so`` (C ABI in ``include/pmgfr.h``);
``paper_1908_03972_amd.api`` is its thin Python binding (import it explicitly: it needs torch
and loads the library). ``paper_1908_03972_amd.esdirk`` holds the published ESDIRK tableaux
and the time-step driver built on ``esdirk_stage_solve``.
"""
__all__ = ["api", "esdirk", "build"]
