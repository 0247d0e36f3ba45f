"""MI355X-native 3D complex DFT (slab, pencil and volumetric schedules).

The HIP library and its ctypes binding load lazily: importing this package
does not touch the GPU.  Use ``paper_1904_10119_amd.dft3d`` for the binding
and ``paper_1904_10119_amd.inputs`` for the seeded synthetic inputs.
"""
__all__ = ["dft3d", "inputs"]
