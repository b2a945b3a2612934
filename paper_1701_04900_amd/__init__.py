"""MI355X-native hot path of the fixed-stepsize SCA block method (AsyFLEXA).

The compute path lives in ``libsca.so`` (hand-written HIP for gfx950 behind a
C ABI declared in ``include/sca.h``); ``paper_1701_04900_amd.sca`` is its thin
ctypes binding and ``paper_1701_04900_amd.inputs`` draws seeded workloads.
Nothing is loaded at import time; the binding raises when the library is absent.
"""
__all__ = ["sca", "inputs"]
