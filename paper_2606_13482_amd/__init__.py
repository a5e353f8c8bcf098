"""Dense EFIE method of moments on one AMD MI355X (gfx950).

`paper_2606_13482_amd.bie` is the ctypes binding of the C-ABI library
`libbie.so` (declared in include/bie.h); `paper_2606_13482_amd.inputs` holds
seeded synthetic meshes and plane waves.  Importing the package loads
nothing; the library is loaded on first use of `bie`.
"""
__version__ = "0.1.0"
