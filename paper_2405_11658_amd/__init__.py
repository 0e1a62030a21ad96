"""MI355X-native dynamic Leiden (Static / ND / DS / DF) community detection.

The compute path is the HIP library ``libleiden_hip.so`` (C-ABI declared in
``include/leiden.h``); ``paper_2405_11658_amd.leiden`` is its thin Python
binding.  Importing this package loads nothing: the binding is imported on
first attribute access, so the input generators (``paper_2405_11658_amd.inputs``)
can be used without the library.
"""
__all__ = ["leiden", "inputs"]


def __getattr__(name):
    if name in ("leiden", "inputs"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
