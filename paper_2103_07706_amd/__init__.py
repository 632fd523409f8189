"""MI355X-native phase-averaged shallow-water right-hand side.

The compute path lives in the HIP/C++ shared library ``libpa.so`` built from
``csrc/`` (C ABI declared in ``include/pa.h``); ``pa`` is its thin ctypes
binding.  Importing this package loads nothing: the library is opened on
first use and a missing library is an error, never a fallback.
"""
