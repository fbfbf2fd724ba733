"""Batched MPS TE-PAI on one MI355X (gfx950).

The computation lives in libtepai.so (HIP kernels behind the C ABI of
include/tepai.h); this package is a thin ctypes binding whose functions carry
the C names.  PyTorch only provides device memory and streams.
"""
from ._lib import (Batch, Handle, ProblemStruct, TepaiError, load, tepai_batch_create,
                   tepai_batch_destroy, tepai_batch_evolve, tepai_batch_observe,
                   tepai_batch_read_mps, tepai_batch_stats, tepai_pai_table, tepai_reduce, tepai_run,
                   tepai_sample_circuits, tepai_validate, tepai_workspace_size)

__all__ = ["Batch", "Handle", "ProblemStruct", "TepaiError", "load", "tepai_batch_create",
           "tepai_batch_destroy", "tepai_batch_evolve", "tepai_batch_observe",
           "tepai_batch_read_mps", "tepai_batch_stats", "tepai_pai_table", "tepai_reduce", "tepai_run",
           "tepai_sample_circuits", "tepai_validate", "tepai_workspace_size"]
