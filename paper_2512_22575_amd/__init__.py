"""MI355X (gfx950) SMPC plan step: HIP kernels behind a C ABI, with a ctypes binding.

``paper_2512_22575_amd.smpc`` binds ``libsmpc.so`` (see ``include/smpc.h``);
``paper_2512_22575_amd.build`` compiles it in-tree.
"""
__all__ = ["smpc", "build"]
