"""MI355X (gfx950) multi-string BWT merge and FMD-index queries.

The computation lives in librb3.so (HIP kernels behind the C ABI declared in
include/rb3.h); ``rb3`` is its ctypes binding.
"""
from .rb3 import (Index, RB3Error, TorchAllocator, rb3_build, rb3_clone, rb3_count, rb3_export,  # noqa: F401
                  rb3_import, rb3_info, rb3_merge, rb3_merge_stats, rb3_prof_enable, rb3_prof_read,
                  rb3_prof_reset, rb3_smem, SMEM_DTYPE)
