"""MI355X (gfx950) pyramid wavefront sensor: HIP kernels behind a C ABI.

``pwfs`` binds the forward model and slope stage (``libpwfs.so``);
``build`` compiles the library in-tree with hipcc.
"""

__all__ = ["pwfs", "build"]
