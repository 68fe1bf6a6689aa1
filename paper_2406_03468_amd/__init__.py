"""MI355X (gfx950) FOSSILS / SPIR least-squares solvers: HIP kernels behind a C ABI.

The compute path is ``libfossils.so`` (built from ``csrc/`` by ``paper_2406_03468_amd.build``);
``binding`` marshals torch device tensors into its C entry points (include/fossils.h).
"""

__all__ = ["binding", "build"]
