"""MI355X-native discrete-velocity Boltzmann-BGK hot path (arXiv 2308.06196).

The compute path is the C-ABI library ``libbgk.so`` (hand-written HIP for
gfx950); ``bgk`` is its thin ctypes binding. Importing the package loads
nothing: the library is opened on first use and raises if it is missing.
"""
