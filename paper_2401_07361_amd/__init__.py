"""MI355X (gfx950) spherical tree code for the barotropic vorticity equation.

The computation lives in the HIP library ``libstc.so`` (C ABI in
``include/stc.h``); ``paper_2401_07361_amd.stc`` is its Python binding.
Build it with ``python -m paper_2401_07361_amd.build``.
"""

__all__ = ["stc", "build"]
