"""Joint-cut hybrid Schroedinger-Feynman simulation on AMD Instinct MI355X.

The work happens in libhsf (HIP kernels for gfx950 plus a C++ planner behind
the C ABI of include/hsf.h).  This package marshals arguments: circuits go in
as host structs, device buffers are torch tensors, and the stream is torch's
current stream.  Functions keep the C names (hsf_plan, hsf_run_paths, ...);
`Plan` bundles them.
"""
from .hsf import (Amplitudes, Batch, Plan, ProbabilityMass, hsf_amplitudes_bitstrings, hsf_amplitudes_full, hsf_amplitudes_full_noalloc,
                  hsf_backward, hsf_loss,
                  hsf_find_blocks, hsf_norm2, hsf_plan, hsf_run_paths, hsf_run_paths_rows, hsf_split_operands, hsf_workspace_size,
                  joint_blocked)
from ._lib import HsfError

__all__ = ["Amplitudes", "Batch", "Plan", "ProbabilityMass", "HsfError", "hsf_plan", "hsf_find_blocks", "joint_blocked",
           "hsf_run_paths", "hsf_run_paths_rows", "hsf_amplitudes_full", "hsf_amplitudes_full_noalloc", "hsf_split_operands", "hsf_amplitudes_bitstrings", "hsf_norm2", "hsf_backward", "hsf_loss",
           "hsf_workspace_size"]
