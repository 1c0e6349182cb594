"""MI355X-native dimension-split wave-propagation step (CUDACLAW method).

The compute path is the HIP library ``libclaw.so`` behind the C ABI declared in
``include/claw.h``; ``paper_1805_08846_amd.claw`` is its ctypes binding and
loads the library when imported.  ``paper_1805_08846_amd.inputs`` builds the
seeded synthetic workloads and needs no GPU library.
"""
