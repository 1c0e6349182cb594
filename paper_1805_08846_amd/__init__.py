"""MI355X-native dimension-split wave-propagation step (CUDACLAW method).

The compute path is the HIP library ``libclaw.so`` behind the C ABI declared in
``include/claw.h``; ``paper_1805_08846_amd.claw`` is its ctypes binding.  The
binding is imported lazily so that the input generators can be used without a
GPU library present.
"""
__all__ = ["claw", "inputs"]


def __getattr__(name):
    if name == "claw":
        from . import claw as _claw
        return _claw
    raise AttributeError(name)
