"""MI355X (gfx950) ground-state AFQMC field-update sweep.

The compute path is the HIP library libpqmc.so built from csrc/ (C ABI in
include/pqmc.h).  This package only marshals arguments to it; PyTorch
supplies the device workspace and the stream.  There is no CPU fallback:
importing `Chain` without the built library raises ImportError.
"""
from .binding import (Chain, Scheme, PQMCError, load_library, library_path,  # noqa: F401
                      EXPORTED_SYMBOLS, MAX_BATCH, batch_sweep, batch_forward_window,
                      multi_sweep, workspace_bytes, SocChain, soc_workspace_bytes,
                      soc_batch_sweep, soc_batch_forward_window)

__all__ = ["Chain", "Scheme", "PQMCError", "load_library", "library_path", "EXPORTED_SYMBOLS",
           "MAX_BATCH", "batch_sweep", "batch_forward_window", "multi_sweep", "workspace_bytes", "SocChain",
           "soc_workspace_bytes", "soc_batch_sweep", "soc_batch_forward_window"]
