"""gedmg: MI355X-native gradient-enhanced damage hot path (HIP kernels behind a C ABI).

`gedmg` holds the ctypes binding of libgedmg.so; `build` compiles it for gfx950.
"""
