"""MI355X (gfx950) Gotoh H/E/F alignment: NW global, SW local and X-drop
seed extension under full / static-band / X-drop pruning.

The compute path is the HIP library ``libaln_hip.so`` behind the C ABI in
``include/aln.h``; ``paper_2607_06225_amd.aln`` is its thin ctypes binding.
``paper_2607_06225_amd.workloads`` builds seeded synthetic inputs.
"""
__all__ = ["aln", "workloads"]
