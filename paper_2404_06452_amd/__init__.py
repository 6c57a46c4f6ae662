"""MI355X-native batched response-time analysis of the PAAM admission test.

``_paam`` is the ctypes binding of libpaam (include/paam.h); ``chaingen`` the
seeded input generator; ``build`` compiles both in-tree.
"""
