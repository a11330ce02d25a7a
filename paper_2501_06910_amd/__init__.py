"""MI355X (gfx950) multi-component error-bounded compressor for values on
unstructured triangle and tetrahedral meshes.

The compute path is the HIP library ``libmc.so`` (C ABI in include/mc.h);
``paper_2501_06910_amd.mc`` is its Python binding.  Build with
``python -m paper_2501_06910_amd.build``.
"""
__all__ = ["mc", "build"]
