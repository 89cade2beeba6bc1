"""MI355X (gfx950) implementation of the intra-query parallel graph search of Speed-ANN
(arXiv 2201.13007).  The kernels live in libspeedann.so (C ABI: include/speedann.h);
``binding`` marshals PyTorch device tensors into it and ``synth`` generates the seeded
workloads.  Submodules load lazily so that the generators import without a GPU."""

__all__ = ["binding", "synth"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
