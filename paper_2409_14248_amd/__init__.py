"""HRKAN physics-informed training step on MI355X (gfx950).

`hrkan` is the binding of the C ABI in include/hrkan.h (libhrkan.so, built by
`python -m paper_2409_14248_amd.build_lib`); `workloads` draws the seeded
synthetic inputs.
"""
from . import workloads  # noqa: F401

__all__ = ["hrkan", "workloads", "build_lib"]


def __getattr__(name):
    if name in ("hrkan", "build_lib"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
