"""hipmr -- run-time generated, fused elementwise and map-reduce kernels for
the AMD Instinct MI355X (gfx950), after the programming model of
Kloeckner et al., "GPU Scripting and Code Generation with PyCUDA".

The compute path is libhipmr.so (C ABI, include/hipmr.h): hand-written HIP
templates specialised and compiled at run time with hipRTC, cached by source
hash.  This package is its thin Python binding; PyTorch provides device
memory and streams only.
"""

from .hipmr import (JOB_NAMES, CFG_FORCE_SCALAR, CFG_SEG_GLOBAL, CFG_TUNED, Graph, Server, autotune_reduce, autotune_segmented,
                    reduce_segmented, segmented_workspace_bytes, scan, scan_workspace_bytes, CFG_NONTEMPORAL, CFG_TEMPORAL, BudgetError, CompileError,
                    ElementwiseKernel, HipError, HipmrError, InvalidError, Kernel, LaunchConfig,
                    MismatchError, ParseError, ReductionKernel, UnsupportedError, WorkspaceError,
                    cache_drop_memory, cache_stats, compile, elementwise, lib, prepare_reduce,
                    reduce, reduce_compensated, norm2, reduce_workspace_bytes, selftest_compile,
                    sha256_hex, torch_dtype)

__all__ = ["ElementwiseKernel", "ReductionKernel", "Kernel", "compile", "elementwise", "reduce",
           "reduce_compensated", "norm2", "reduce_segmented", "segmented_workspace_bytes", "scan",
           "scan_workspace_bytes",
           "autotune_segmented", "autotune_reduce", "Graph", "Server", "JOB_NAMES",
           "prepare_reduce", "reduce_workspace_bytes", "cache_stats", "cache_drop_memory",
           "sha256_hex", "selftest_compile", "lib", "torch_dtype", "LaunchConfig",
           "CFG_NONTEMPORAL", "CFG_TEMPORAL", "CFG_FORCE_SCALAR", "CFG_SEG_GLOBAL", "CFG_TUNED",
           "HipmrError", "InvalidError",
           "ParseError", "CompileError", "HipError", "MismatchError", "UnsupportedError",
           "BudgetError", "WorkspaceError"]
