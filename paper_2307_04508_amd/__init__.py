"""MI355X-native LT-AC G0W0 hot path (Laplace-transformed polarizability,
screening, diagonal self-energy, Pade continuation) behind the C ABI of
``include/gwlt.h``.  ``gwlt`` is the Python binding of that ABI; it loads
the in-tree ``libgwlt.so`` built by ``build.py`` and raises if it is missing.
"""
