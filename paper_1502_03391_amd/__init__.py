"""MI355X (gfx950) fast JOFC: HIP kernels behind a C ABI (include/fjofc.h).

``paper_1502_03391_amd.fjofc`` is the ctypes binding; ``build`` compiles
the library.  Importing the package loads nothing.
"""
__all__ = ["fjofc", "build"]
