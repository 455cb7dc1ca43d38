"""MI355X-native short-characteristics radiation transport solver (arXiv 2107.08145).

The solver itself is the HIP library `librts.so` behind the C ABI declared in
`include/rts.h`; `paper_2107_08145_amd.rts` is its thin ctypes binding and
`paper_2107_08145_amd.inputs` the seeded synthetic problem generator.
"""
__all__ = ["inputs", "rts"]
