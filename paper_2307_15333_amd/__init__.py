"""MI355X-native octree volume renderer of the Dynamic PlenOctree method.

``core`` (trees, ray batches, the autograd function) loads the HIP library
``libdot.so``; ``synth`` holds seeded input generators and needs only NumPy.
Submodules are imported lazily so that the generators stay usable without a
built library.
"""

__all__ = ["core", "synth", "serve"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
