"""MI355X-native immersed-boundary (IB-GM) time-step library.

The compute path is the C-ABI library ``libibgm.so`` (hand-written HIP for
gfx950); ``paper_1305_3976_amd.ibgm`` is its thin ctypes binding and
``paper_1305_3976_amd.inputs`` builds seeded synthetic workloads.  Importing
the package does not load the library: ``ibgm`` does, and fails loudly when it
is missing.
"""
__all__ = ["inputs", "ibgm"]
