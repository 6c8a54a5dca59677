"""MI355X-native spherical curvelet transform (spin 0, McEwen-Wiaux sampling).

The transform runs in hand-written HIP kernels for gfx950 behind a C ABI
(``include/curvelet.h``); ``paper_1511_05578_amd.api`` is the thin ctypes
binding.  Importing this package does not load the native library; the first
call into ``api`` does, and raises if it has not been built.
"""
