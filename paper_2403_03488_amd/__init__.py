"""BM3D stage of the nonlocal + lightweight-CNN denoiser, native on MI355X (gfx950).

The compute path is the HIP library built from ``csrc/`` behind the C ABI in
``include/bm3d.h``; ``bm3d`` is its thin Python binding (argument marshalling
only).  Import ``paper_2403_03488_amd.bm3d`` to load the library.
"""
