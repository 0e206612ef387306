"""Python binding of the reduced-basis entry points (fixed excitation number,
even mirror parity; Sec. III.A).  Argument marshalling only: the tables are
built by kg_pe_build and every product runs in libkgrape.so's kernels."""

from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import KG_GRAD_CENTRED, KG_GRAD_FIRST_ORDER, KG_GRAD_QUADRATURE, KG_GRAD_ZEROTH, KgPe
from .api import XXZ, GrapeResult, Krylov, _f64, _ptr, _stream, prec_of


def pe_dim(L: int, K: int) -> int:
    d = int(_lib.load().kg_pe_dim(int(L), int(K)))
    if d == 0:
        raise ValueError(_lib.last_error())
    return d


def pe_tables_host(L: int, K: int) -> dict:
    """The tables as kg_pe_tables_host writes them (host memory, no device):
    binom (33 x 33), reps (dim,), ranks (dim,), index (C(L, K),) and, when the
    basis has a neighbour table, slot_counts (slices,) and neighbors
    (slices, L - 1, 64)."""
    lib = _lib.load()
    nb = int(lib.kg_pe_tables_bytes(int(L), int(K)))
    if nb == 0:
        raise ValueError(_lib.last_error())
    buf = np.zeros(nb, dtype=np.uint8)
    _lib.check("kg_pe_tables_host", lib.kg_pe_tables_host(
        int(L), int(K), ctypes.c_void_p(buf.ctypes.data), nb))
    dim = pe_dim(L, K)
    off_reps = 4608
    R = (4 * dim + 255) // 256 * 256
    off_ranks = off_reps + R
    off_index = off_ranks + R
    from math import comb
    out = {"binom": buf[:4 * 33 * 33].view(np.uint32).reshape(33, 33),
           "reps": buf[off_reps:off_reps + 4 * dim].view(np.uint32),
           "ranks": buf[off_ranks:off_ranks + 4 * dim].view(np.uint32),
           "index": buf[off_index:off_index + 4 * comb(L, K)].view(np.int32)}
    off_cnt = off_index + (4 * comb(L, K) + 255) // 256 * 256
    ns = (dim + 63) // 64
    if off_cnt < nb:
        off_nbr = off_cnt + (4 * ns + 255) // 256 * 256
        out["slot_counts"] = buf[off_cnt:off_cnt + 4 * ns].view(np.uint32)
        out["neighbors"] = buf[off_nbr:nb].view(np.uint32).reshape(ns, L - 1, 64)
    return out


class ReducedBasis:
    """Device tables of the K-excitation, even-parity basis of L spins."""

    def __init__(self, L: int, K: int, device=None):
        lib = _lib.load()
        nb = int(lib.kg_pe_tables_bytes(int(L), int(K)))
        if nb == 0:
            raise ValueError(_lib.last_error())
        self.buf = torch.empty(nb + 256, dtype=torch.uint8, device=device or torch.device("cuda"))
        off = (-self.buf.data_ptr()) % 256
        self.pe = KgPe()
        _lib.check("kg_pe_build", lib.kg_pe_build(
            int(L), int(K), ctypes.c_void_p(self.buf.data_ptr() + off), nb, ctypes.byref(self.pe)))
        self.L, self.K, self.dim = int(L), int(K), int(self.pe.dim)

    def ref(self):
        return ctypes.byref(self.pe)


class ReducedWorkspace:
    """Device scratch of the reduced-basis Krylov calls and sweeps."""

    def __init__(self, B: ReducedBasis, k: Krylov, dtype: torch.dtype, device=None,
                 extended: bool = False):
        self.nbytes = int(_lib.load().kg_pe_workspace_bytes(B.ref(), ctypes.byref(k.c()),
                                                            prec_of(dtype), 1 if extended else 0))
        if self.nbytes == 0:
            raise ValueError(_lib.last_error())
        self.buf = torch.empty(self.nbytes + 256, dtype=torch.uint8,
                               device=device or torch.device("cuda"))
        off = (-self.buf.data_ptr()) % 256
        self.ptr = ctypes.c_void_p(self.buf.data_ptr() + off)
        self.key = (B.L, B.K, k.m, dtype, extended)


def _rvec(t: torch.Tensor, B: ReducedBasis, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if t.numel() != B.dim or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous vector of dim = {B.dim} amplitudes")
    return t


def _rws(ws, B, k, dtype, device, extended=False):
    if ws is None or ws.key[:4] != (B.L, B.K, k.m, dtype) or (extended and not ws.key[4]):
        ws = ReducedWorkspace(B, k, dtype, device, extended)
    return ws


def pe_states(B: ReducedBasis, N: int, ckpt_every: int, dtype, device=None) -> torch.Tensor:
    nb = int(_lib.load().kg_pe_states_bytes(B.ref(), int(N), int(ckpt_every), prec_of(dtype)))
    if nb == 0:
        raise ValueError(_lib.last_error())
    esz = 16 if dtype == torch.complex128 else 8
    return torch.empty(nb // esz, dtype=dtype, device=device or torch.device("cuda"))


def xxz_pe_apply(h: XXZ, B: ReducedBasis, u: float, v: torch.Tensor,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """w = (H0 + u Hc) v in the reduced basis."""
    _rvec(v, B, v.dtype, "v")
    w = torch.empty_like(v) if out is None else _rvec(out, B, v.dtype, "out")
    _lib.check("xxz_pe_apply", _lib.load().xxz_pe_apply(
        ctypes.byref(h.c()), B.ref(), float(u), prec_of(v.dtype), _ptr(v), _ptr(w), _stream()))
    return w


def krylov_expv_pe(h: XXZ, B: ReducedBasis, u: float, t: float, v: torch.Tensor, k: Krylov,
                   out: Optional[torch.Tensor] = None, workspace: Optional[ReducedWorkspace] = None,
                   m_eff: Optional[torch.Tensor] = None) -> torch.Tensor:
    """exp(-i t (H0 + u Hc)) v in the reduced basis (out may be v)."""
    _rvec(v, B, v.dtype, "v")
    w = torch.empty_like(v) if out is None else _rvec(out, B, v.dtype, "out")
    ws = _rws(workspace, B, k, v.dtype, v.device)
    _lib.check("krylov_expv_pe", _lib.load().krylov_expv_pe(
        ctypes.byref(h.c()), B.ref(), float(u), float(t), ctypes.byref(k.c()), prec_of(v.dtype),
        _ptr(v), _ptr(w), ws.ptr, ws.nbytes, _ptr(m_eff), _stream()))
    return w


def grape_forward_pe(h: XXZ, B: ReducedBasis, u: torch.Tensor, dt: float, k: Krylov,
                     psi0: torch.Tensor, target: torch.Tensor, ckpt_every: int = 0,
                     states: Optional[torch.Tensor] = None,
                     workspace: Optional[ReducedWorkspace] = None) -> GrapeResult:
    dtype = psi0.dtype
    _rvec(psi0, B, dtype, "psi0")
    _rvec(target, B, dtype, "target")
    N = u.numel()
    _f64(u, N, "u")
    if states is None:
        states = pe_states(B, N, ckpt_every, dtype, psi0.device)
    ws = _rws(workspace, B, k, dtype, psi0.device)
    F = torch.empty((), dtype=torch.float64, device=psi0.device)
    beta = torch.empty(2, dtype=torch.float64, device=psi0.device)
    _lib.check("grape_forward_pe", _lib.load().grape_forward_pe(
        ctypes.byref(h.c()), B.ref(), _ptr(u), N, float(dt), ctypes.byref(k.c()), prec_of(dtype),
        _ptr(psi0), _ptr(target), _ptr(F), _ptr(beta), _ptr(states), int(ckpt_every), ws.ptr,
        ws.nbytes, _stream()))
    return GrapeResult(F=F, beta=beta, grad=None, states=states)


_VARIANTS = {"zeroth": KG_GRAD_ZEROTH, "centred": KG_GRAD_CENTRED,
             "first_order": KG_GRAD_FIRST_ORDER, "quadrature": KG_GRAD_QUADRATURE}


def grape_gradient_pe(h: XXZ, B: ReducedBasis, u: torch.Tensor, dt: float, k: Krylov,
                      psi0: torch.Tensor, target: torch.Tensor, ckpt_every: int = 0,
                      variant: str = "zeroth", nodes: int = 0,
                      states: Optional[torch.Tensor] = None, states_valid: bool = False,
                      beta: Optional[torch.Tensor] = None,
                      workspace: Optional[ReducedWorkspace] = None,
                      F: Optional[torch.Tensor] = None,
                      grad: Optional[torch.Tensor] = None) -> GrapeResult:
    """Fidelity and gradient in the reduced basis; `variant` is "zeroth",
    "centred", "first_order" or "quadrature" (with `nodes`)."""
    dtype = psi0.dtype
    _rvec(psi0, B, dtype, "psi0")
    _rvec(target, B, dtype, "target")
    N = u.numel()
    _f64(u, N, "u")
    dev = psi0.device
    if states is None:
        if states_valid:
            raise ValueError("states_valid needs the states of grape_forward_pe")
        states = pe_states(B, N, ckpt_every, dtype, dev)
    if states_valid and beta is None:
        raise ValueError("states_valid needs beta from grape_forward_pe")
    v = _VARIANTS[variant]
    ws = _rws(workspace, B, k, dtype, dev, extended=v in (KG_GRAD_FIRST_ORDER, KG_GRAD_QUADRATURE))
    if F is None:
        F = torch.empty((), dtype=torch.float64, device=dev)
    if beta is None:
        beta = torch.empty(2, dtype=torch.float64, device=dev)
    if grad is None:
        grad = torch.empty(N, dtype=torch.float64, device=dev)
    _f64(grad, N, "grad")
    _lib.check("grape_gradient_pe", _lib.load().grape_gradient_pe(
        ctypes.byref(h.c()), B.ref(), _ptr(u), N, float(dt), ctypes.byref(k.c()), prec_of(dtype),
        _ptr(psi0), _ptr(target), _ptr(F), _ptr(beta), _ptr(grad), _ptr(states), int(ckpt_every),
        1 if states_valid else 0, v, int(nodes), ws.ptr, ws.nbytes, _stream()))
    return GrapeResult(F=F, beta=beta, grad=grad, states=states)


__all__ = ["ReducedBasis", "ReducedWorkspace", "pe_dim", "pe_tables_host", "pe_states",
           "xxz_pe_apply", "krylov_expv_pe", "grape_forward_pe", "grape_gradient_pe"]
