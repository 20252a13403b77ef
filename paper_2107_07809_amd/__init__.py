"""MI355X engine for the register-state dataflow analysis of GCN kernels
(decompilation method of Mihajlenko, Lukin & Stankevich).

The product is libdc.so (HIP kernels for gfx950 behind the C ABI in
include/dc.h); ``paper_2107_07809_amd.dc`` is its ctypes binding.  Importing
this package loads nothing; ``dc.lib()`` loads the library and fails loudly
when it has not been built.
"""
