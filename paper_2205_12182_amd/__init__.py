"""MI355X (gfx950) non-orthogonal local submatrix method: HIP kernels behind a C ABI.

    from paper_2205_12182_amd import _lib, runner

`_lib` mirrors include/nolsm.h (ctypes); `runner.Runner` drives it over a whole
block-sparse instance with PyTorch device memory.  The library must be built
(`python -m paper_2205_12182_amd.build`); nothing here computes on the CPU.
"""
