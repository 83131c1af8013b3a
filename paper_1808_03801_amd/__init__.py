"""MI355X-native USP-ESBGK particle solver (arXiv 1808.03801).

The hot path lives in the HIP library ``libusp.so`` (``csrc/``), reached
through the thin ctypes binding in ``paper_1808_03801_amd.usp``.  Importing
this package loads nothing; the binding raises if the library is missing.
"""
