"""Helpers shared by the GPU tests (no method arithmetic here)."""

import contextlib
import os

import numpy as np
import torch

import paper_2010_03598_amd as kg

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None
C128 = torch.complex128
C64 = torch.complex64


def dev_vec(x, dtype=C128):
    return torch.tensor(np.asarray(x), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


@contextlib.contextmanager
def tile_bits(tb):
    """Force the tile size of the tiled kernels (exercises every tiling variant)."""
    old = os.environ.get("KG_TILE_BITS")
    os.environ["KG_TILE_BITS"] = str(tb)
    try:
        yield
    finally:
        if old is None:
            del os.environ["KG_TILE_BITS"]
        else:
            os.environ["KG_TILE_BITS"] = old


@contextlib.contextmanager
def tiled_only():
    """Run Krylov calls through the tiled multi-launch passes even where the
    one-block form would apply (small vectors)."""
    old = os.environ.get("KG_NO_FUSED")
    os.environ["KG_NO_FUSED"] = "1"
    try:
        yield
    finally:
        if old is None:
            del os.environ["KG_NO_FUSED"]
        else:
            os.environ["KG_NO_FUSED"] = old


def xxz_of(c):
    return kg.XXZ(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
