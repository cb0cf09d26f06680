"""MI355X-native GPU filtering stage of a multi-tiered IVF-PQ index.

The search path (probe, distance table, ID gather + dedup, ADC scan, top-n,
exact re-rank) runs as hand-written HIP kernels for gfx950 behind the C ABI in
``include/ann.h``; ``paper_2409_16576_amd.ann`` is its thin ctypes binding.
"""
__all__ = ["inputs", "workloads", "builder", "ann"]
