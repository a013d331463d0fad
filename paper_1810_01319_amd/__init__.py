"""MI355X-native hot path of an array-of-octrees AMR hydro step (Enzo-P/Cello).

The compute runs in the HIP library ``libamr.so`` behind the C ABI of
``include/amr.h``; ``mesh.Mesh`` marshals torch device tensors into it.
Import of this package is light: the library is loaded on first use.
"""
__all__ = ["Mesh"]


def __getattr__(name):
    if name == "Mesh":
        from .mesh import Mesh

        return Mesh
    raise AttributeError(name)
