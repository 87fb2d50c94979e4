"""FORA approximate single-source Personalized PageRank on MI355X (gfx950).

The method runs in the HIP library ``libfora.so`` (see ``include/fora.h``);
``fora`` is its Python binding. Importing ``fora`` fails if the library has
not been built (``__graft_entry__.build()``): there is no CPU fallback.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfora.so")


def load():
    """Import the binding (raises ImportError if the HIP library is missing)."""
    from . import fora
    return fora
