"""MI355X-native fast weighted bit-flipping (FWBF) LDPC decoder.

The compute path is the HIP library ``libfwbf.so`` (``csrc/``); ``fwbf`` is
its thin ctypes binding.  Importing the package loads nothing native; the
binding loads the library on first use and raises if it is missing.
"""
