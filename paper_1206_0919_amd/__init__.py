"""MI355X-native relativistic SHASTA time step (arXiv:1206.0919).

The compute path is the C-ABI library ``libshasta.so`` (hand-written HIP
kernels for gfx950, see ``csrc/``); ``binding`` exposes it to Python with the
same function names.  Importing this package loads nothing: the library is
loaded on first use of :mod:`paper_1206_0919_amd.binding`.
"""
__all__ = ["binding", "inputs"]
