"""3DGStream Stage-1 hot path on MI355X (gfx950).

`gs3`    ctypes binding of libgs3.so (the C ABI in include/gs3.h)
`synth`  seeded synthetic scenes, cameras, motion fields, NTC initial parameters
`train`  Stage-1 training loops (NTC and direct optimisation) on the C ABI
`build`  hipcc build of libgs3.so
"""
