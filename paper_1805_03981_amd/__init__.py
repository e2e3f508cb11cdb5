"""dgw: matrix-free DG acoustics on curved quad/hex meshes for MI355X (gfx950).

The solver is the HIP library libdgw.so behind the C ABI of include/dgw.h;
`paper_1805_03981_amd.binding` is its Python binding (ctypes; PyTorch for
device memory and streams).  Build with `python -m paper_1805_03981_amd.build`.
"""
__all__ = ["binding", "build"]
