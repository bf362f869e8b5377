"""MI355X-native likelihood for time-dependent four-body amplitude fits
(D0 -> K+ pi- pi+ pi-, arXiv:1702.06735).

The computation runs in the HIP library ``libmixamp.so`` (``csrc/``); the
``mixamp`` module is its ctypes binding and ``inputs`` generates seeded
synthetic events. Importing the package loads nothing; the library is loaded
on first use and raises if it is missing.
"""
