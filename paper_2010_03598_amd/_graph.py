"""Guard for HIP graph captures made through torch.cuda.graph."""

from __future__ import annotations

import contextlib
import gc

import torch


@contextlib.contextmanager
def capture_guard():
    """Collect Python garbage before a capture and keep the collector off until
    it ends.  A collection inside the capture could free device memory of dead
    objects (tensors, graphs) while the stream is capturing, which the runtime
    refuses; the error then surfaces in a destructor and ends the process."""
    torch.cuda.synchronize()
    gc.collect()
    was_enabled = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was_enabled:
            gc.enable()
