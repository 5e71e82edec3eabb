"""Full-sky pixel-relative Taylor lensing on MI355X (gfx950).

The compute path is the HIP library ``libtaylens.so`` (C ABI in
``include/taylens.h``); ``paper_1307_0719_amd.taylens`` is its Python
binding.  Submodules are imported lazily so that the input generator
(``skygen``) can be used without the GPU library.
"""

__all__ = ["taylens", "skygen", "build"]


def __getattr__(name):
    import importlib

    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
