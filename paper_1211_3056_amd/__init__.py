"""MI355X-native hard-to-round case search (HIP kernels behind a C ABI).

Modules: _lib (ctypes binding of libhrsearch.so), api (buffer handling),
prep (host tables, windows, thresholds), pipeline (one job end to end),
build (compiles the library for gfx950).
"""
