"""MI355X (gfx950) implementation of the GPU-accelerated kernel-free boundary
integral (KFBI) time-stepping method for the heat, wave and Schroedinger
equations on irregular 2-D domains.

The compute path is the HIP library libkfbi.so (sources in csrc/, C ABI in
include/kfbi.h); `paper_2404_14864_amd.kfbi` is its thin ctypes binding and
`paper_2404_14864_amd.build` compiles it for gfx950.
"""
