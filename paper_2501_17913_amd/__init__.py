"""MI355X-native tensor jump method (TJM): the per-trajectory TJM step of
arXiv:2501.17913 as HIP kernels for CDNA4 behind a C ABI (include/tjm.h).

Modules
-------
tjm      ctypes binding of libtjm.so (argument marshalling only)
models   builders of the inputs the C ABI takes: MPOs, jump sets, observables,
         product states
build    compiles libtjm.so for gfx950
"""
