"""MI355X (gfx950) library for variational photoacoustic tomography reconstruction
with preconditioned PDHGM (arXiv:1707.02245).

The compute path is the HIP library libpat.so behind the C ABI in include/pat.h;
`paper_1707_02245_amd.pat` is its Python binding. Import of the binding fails
loudly when the library has not been built.
"""

__all__ = ["pat", "build"]
