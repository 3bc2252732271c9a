"""MI355X-native detection of topological changes in dynamic lattice Voronoi
diagrams (Bernaschi, Lulli, Sbragaglia, arXiv:1607.00908).

* ``dv``     -- binding of the HIP library libdv.so (C ABI in include/dv.h)
* ``serve``  -- continuous batching of frames from many streams (groups)
* ``synth``  -- seeded synthetic workloads (input generation only)

Submodules are imported on demand so that the workload generators can be used
without loading the GPU library.
"""

__all__ = ["dv", "serve", "synth"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
