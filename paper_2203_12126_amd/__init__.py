"""MI355X-native IBDL hot path (Leathers & Guy, Immersed Boundary Double Layer method).

The compute path lives in the HIP library ``libibdl.so`` (C-ABI, ``include/ibdl.h``);
``paper_2203_12126_amd.ibdl`` is its thin Python binding and
``paper_2203_12126_amd.workloads`` holds the seeded synthetic inputs.  Importing
the package itself loads nothing.
"""
__all__ = ["ibdl", "workloads"]
