"""MI355X (gfx950) implementation of the Disentangled 4D Gaussian Splatting render path.

Submodules:
    inputs   -- seeded synthetic scenes, cameras and request streams
    binding  -- ctypes binding of the C-ABI library libd4dgs.so (hand-written HIP)
    render   -- PyTorch-facing wrappers: render(), the autograd Function, the server

The binding is imported on first use so that the inputs module can be used on a
machine without the built library; every compute entry point fails loudly when the
library is missing.
"""
__all__ = ["inputs", "binding", "render"]
__version__ = "0.1.0"


def __getattr__(name):
    if name in ("binding", "render"):
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
