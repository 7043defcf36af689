"""MI355X (gfx950) renderer for Sparse Neural Radiance Grids (SNeRG, arXiv 2103.14645).

The render path is the HIP library libsnerg.so (C ABI: include/snerg.h);
`snerg` is its Python binding and `autograd` wraps the forward/backward pair
as a torch.autograd.Function.
"""
from . import snerg  # noqa: F401
