"""Python binding of the K-GRAPE C ABI (argument marshalling only).

Every entry point has the name of its C counterpart and forwards device
pointers of torch tensors plus torch's current HIP stream; all arithmetic runs
in the HIP kernels of libkgrape.so.  torch supplies device memory and streams.
"""

from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import torch

from . import _lib
from ._lib import KG_C64, KG_C128, KG_HC_SX, KG_HC_SZ, KgKrylov, KgXxz  # noqa: F401


@dataclasses.dataclass(frozen=True)
class XXZ:
    """Open XXZ chain H0 = J sum (SxSx + SySy + Delta SzSz), S = sigma/2, with a
    control operator: S^x on one site (hc_kind=KG_HC_SX) or a sum of S^z
    (KG_HC_SZ).  hc_sites: bit (i-1) set <=> site i (1-based) carries it."""

    L: int
    J: float = 1.0
    Delta: float = 0.5
    hc_kind: int = KG_HC_SX
    hc_sites: int = 1

    @property
    def D(self) -> int:
        return 1 << self.L

    def c(self) -> KgXxz:
        return KgXxz(self.L, self.hc_kind, float(self.J), float(self.Delta), int(self.hc_sites))


@dataclasses.dataclass(frozen=True)
class Krylov:
    """Krylov dimension m, full re-orthogonalisation flag, relative breakdown
    tolerance (0 = 64 unit roundoffs of the vector type)."""

    m: int
    reorth: bool = True
    breakdown_tol: float = 0.0

    def c(self) -> KgKrylov:
        return KgKrylov(int(self.m), 1 if self.reorth else 0, float(self.breakdown_tol))


def prec_of(dtype: torch.dtype) -> int:
    if dtype == torch.complex128:
        return KG_C128
    if dtype == torch.complex64:
        return KG_C64
    raise TypeError(f"state vectors must be complex128 or complex64, not {dtype}")


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _vec(t: torch.Tensor, h: XXZ, dtype: torch.dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if t.numel() != h.D or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous vector of 2^L = {h.D} amplitudes")
    return t


def _f64(t: torch.Tensor, n: int, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA/HIP tensor")
    if t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous vector of {n} values")
    return t


def _ws_bytes(h: XXZ, k: Krylov, dtype: torch.dtype, extended: bool) -> int:
    fn = "kg_extended_workspace_bytes" if extended else "kg_workspace_bytes"
    return int(getattr(_lib.load(), fn)(ctypes.byref(h.c()), ctypes.byref(k.c()), prec_of(dtype)))


class Workspace:
    """Device scratch for krylov_expv / grape_forward / grape_gradient (with
    `extended`, large enough for the quadrature and first-order gradients too)."""

    def __init__(self, h: XXZ, k: Krylov, dtype: torch.dtype, device=None,
                 extended: bool = False):
        self.nbytes = _ws_bytes(h, k, dtype, extended)
        if self.nbytes == 0:
            raise ValueError(_lib.last_error() or "invalid chain or Krylov options")
        self.buf = torch.empty(self.nbytes + 256, dtype=torch.uint8,
                               device=device or torch.device("cuda"))
        off = (-self.buf.data_ptr()) % 256
        self.ptr = ctypes.c_void_p(self.buf.data_ptr() + off)

    def fits(self, h: XXZ, k: Krylov, dtype: torch.dtype, extended: bool = False) -> bool:
        need = _ws_bytes(h, k, dtype, extended)
        return need != 0 and need <= self.nbytes


def states_bytes(h: XXZ, N: int, ckpt_every: int, dtype: torch.dtype) -> int:
    n = int(_lib.load().kg_states_bytes(ctypes.byref(h.c()), N, ckpt_every, prec_of(dtype)))
    if n == 0:
        raise ValueError(_lib.last_error())
    return n


def new_states(h: XXZ, N: int, ckpt_every: int, dtype: torch.dtype, device=None) -> torch.Tensor:
    """State buffer for grape_forward/grape_gradient (vectors of `dtype`)."""
    nb = states_bytes(h, N, ckpt_every, dtype)
    esz = 16 if dtype == torch.complex128 else 8
    return torch.empty(nb // esz, dtype=dtype, device=device or torch.device("cuda"))


def _ws(ws: Optional[Workspace], h: XXZ, k: Krylov, dtype, device,
        extended: bool = False) -> Workspace:
    if ws is None or not ws.fits(h, k, dtype, extended):
        ws = Workspace(h, k, dtype, device, extended)
    return ws


def xxz_apply(h: XXZ, u: float, v: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """w = (H0 + u Hc) v."""
    _vec(v, h, v.dtype, "v")
    w = torch.empty_like(v) if out is None else _vec(out, h, v.dtype, "out")
    _lib.check("xxz_apply", _lib.load().xxz_apply(ctypes.byref(h.c()), float(u), prec_of(v.dtype),
                                                  _ptr(v), _ptr(w), _stream()))
    return w


def krylov_expv(h: XXZ, u: float, t: float, v: torch.Tensor, k: Krylov,
                out: Optional[torch.Tensor] = None, workspace: Optional[Workspace] = None,
                m_eff: Optional[torch.Tensor] = None) -> torch.Tensor:
    """exp(-i t (H0 + u Hc)) v by an m-dimensional Lanczos basis (out may be v)."""
    _vec(v, h, v.dtype, "v")
    w = torch.empty_like(v) if out is None else _vec(out, h, v.dtype, "out")
    ws = _ws(workspace, h, k, v.dtype, v.device)
    if m_eff is not None and (m_eff.dtype != torch.int32 or not m_eff.is_cuda or m_eff.numel() < 1):
        raise TypeError("m_eff must be an int32 CUDA/HIP tensor")
    _lib.check("krylov_expv", _lib.load().krylov_expv(
        ctypes.byref(h.c()), float(u), float(t), ctypes.byref(k.c()), prec_of(v.dtype), _ptr(v),
        _ptr(w), ws.ptr, ws.nbytes, _ptr(m_eff), _stream()))
    return w


@dataclasses.dataclass
class GrapeResult:
    F: torch.Tensor          # () float64, |<f|psi_N>|^2
    beta: torch.Tensor       # (2,) float64, (re, im) of <f|psi_N>
    grad: Optional[torch.Tensor]  # (N,) float64, dF/du_j
    states: torch.Tensor     # forward-state buffer (layout of ckpt_every)


def grape_forward(h: XXZ, u: torch.Tensor, dt: float, k: Krylov, psi0: torch.Tensor,
                  target: torch.Tensor, ckpt_every: int = 0, states: Optional[torch.Tensor] = None,
                  workspace: Optional[Workspace] = None) -> GrapeResult:
    """Forward sweep psi_j = exp(-i dt H_j) psi_{j-1}; beta = <f|psi_N>, F = |beta|^2."""
    dtype = psi0.dtype
    _vec(psi0, h, dtype, "psi0")
    _vec(target, h, dtype, "target")
    N = u.numel()
    _f64(u, N, "u")
    if states is None:
        states = new_states(h, N, ckpt_every, dtype, psi0.device)
    elif states.numel() * states.element_size() < states_bytes(h, N, ckpt_every, dtype):
        raise ValueError("states buffer too small")
    ws = _ws(workspace, h, k, dtype, psi0.device)
    F = torch.empty((), dtype=torch.float64, device=psi0.device)
    beta = torch.empty(2, dtype=torch.float64, device=psi0.device)
    _lib.check("grape_forward", _lib.load().grape_forward(
        ctypes.byref(h.c()), _ptr(u), N, float(dt), ctypes.byref(k.c()), prec_of(dtype), _ptr(psi0),
        _ptr(target), _ptr(F), _ptr(beta), _ptr(states), int(ckpt_every), ws.ptr, ws.nbytes,
        _stream()))
    return GrapeResult(F=F, beta=beta, grad=None, states=states)


def grape_gradient(h: XXZ, u: torch.Tensor, dt: float, k: Krylov, psi0: torch.Tensor,
                   target: torch.Tensor, ckpt_every: int = 0, states: Optional[torch.Tensor] = None,
                   states_valid: bool = False, beta: Optional[torch.Tensor] = None,
                   grad: Optional[torch.Tensor] = None, F: Optional[torch.Tensor] = None,
                   workspace: Optional[Workspace] = None, centred: bool = False,
                   nodes: int = 0, first_order: bool = False) -> GrapeResult:
    """Fidelity and gradient dF/du_j: the zeroth-order gradient of Eq. 5; with
    `centred` its centred variant (the bracket at both ends of each slice,
    averaged; App. B); with `nodes` > 0 the exact piecewise-constant gradient by
    `nodes`-point Gauss-Legendre quadrature inside each slice; with
    `first_order` the first order of the hierarchy of the time-averaged control
    operator (one commutator with H_j).  With states_valid, `states` and `beta`
    must come from grape_forward with the same arguments."""
    if int(bool(centred)) + int(bool(nodes)) + int(bool(first_order)) > 1:
        raise ValueError("centred, nodes and first_order are exclusive")
    dtype = psi0.dtype
    _vec(psi0, h, dtype, "psi0")
    _vec(target, h, dtype, "target")
    N = u.numel()
    _f64(u, N, "u")
    dev = psi0.device
    if states is None:
        if states_valid:
            raise ValueError("states_valid needs the states of grape_forward")
        states = new_states(h, N, ckpt_every, dtype, dev)
    elif states.numel() * states.element_size() < states_bytes(h, N, ckpt_every, dtype):
        raise ValueError("states buffer too small")
    if states_valid and beta is None:
        raise ValueError("states_valid needs beta from grape_forward")
    ws = _ws(workspace, h, k, dtype, dev, extended=bool(nodes) or first_order)
    if F is None:
        F = torch.empty((), dtype=torch.float64, device=dev)
    if beta is None:
        beta = torch.empty(2, dtype=torch.float64, device=dev)
    if grad is None:
        grad = torch.empty(N, dtype=torch.float64, device=dev)
    _f64(grad, N, "grad")
    args = [ctypes.byref(h.c()), _ptr(u), N, float(dt), ctypes.byref(k.c()), prec_of(dtype),
            _ptr(psi0), _ptr(target), _ptr(F), _ptr(beta), _ptr(grad), _ptr(states),
            int(ckpt_every), 1 if states_valid else 0]
    if nodes:
        name = "grape_gradient_quadrature"
        args.append(int(nodes))
    elif first_order:
        name = "grape_gradient_first_order"
    else:
        name = "grape_gradient_centred" if centred else "grape_gradient"
    _lib.check(name, getattr(_lib.load(), name)(*args, ws.ptr, ws.nbytes, _stream()))
    return GrapeResult(F=F, beta=beta, grad=grad, states=states)


@dataclasses.dataclass
class ColumnsResult:
    F: torch.Tensor          # () float64, |beta|^2
    beta: torch.Tensor       # (2,) float64, beta = (1/n) sum_c <w_c|psi_c(T)>
    beta_cols: torch.Tensor  # (n, 2) float64, <w_c|psi_c(T)> per column
    grad: torch.Tensor       # (N,) float64, dF/du_j
    states: torch.Tensor


def grape_gradient_columns(h: XXZ, u: torch.Tensor, dt: float, k: Krylov, psi0s: torch.Tensor,
                           targets: torch.Tensor, ckpt_every: int = 0, centred: bool = False,
                           basis=None, states: Optional[torch.Tensor] = None,
                           workspace=None) -> ColumnsResult:
    """Operator control on a block of columns: F = |(1/n) sum_c <w_c|U(T)|psi_c>|^2
    and its (zeroth-order or centred) gradient.  psi0s, targets: (n, D)
    contiguous tensors of one complex dtype (D = 2^L, or the dimension of
    `basis`, a ReducedBasis)."""
    dtype = psi0s.dtype
    prec = prec_of(dtype)
    if psi0s.dim() != 2 or targets.shape != psi0s.shape or targets.dtype != dtype:
        raise ValueError("psi0s and targets must be (n, D) tensors of the same dtype")
    if not (psi0s.is_cuda and targets.is_cuda and psi0s.is_contiguous() and targets.is_contiguous()):
        raise ValueError("psi0s and targets must be contiguous CUDA/HIP tensors")
    n, D = psi0s.shape
    if D != (h.D if basis is None else basis.dim):
        raise ValueError(f"columns of {D} amplitudes do not match the space")
    N = u.numel()
    _f64(u, N, "u")
    dev = psi0s.device
    lib = _lib.load()
    if basis is None:
        one = states_bytes(h, N, ckpt_every, dtype)
        ws = _ws(workspace, h, k, dtype, dev)
    else:
        from . import reduced
        one = int(lib.kg_pe_states_bytes(basis.ref(), N, int(ckpt_every), prec))
        if one == 0:
            raise ValueError(_lib.last_error())
        ws = reduced._rws(workspace, basis, k, dtype, dev)
    esz = 16 if dtype == torch.complex128 else 8
    if states is None:
        states = torch.empty(n * one // esz, dtype=dtype, device=dev)
    elif states.numel() * states.element_size() < n * one:
        raise ValueError("states buffer too small")
    F = torch.empty((), dtype=torch.float64, device=dev)
    beta = torch.empty(2, dtype=torch.float64, device=dev)
    beta_cols = torch.empty((n, 2), dtype=torch.float64, device=dev)
    grad = torch.empty(N, dtype=torch.float64, device=dev)
    common = [N, float(dt), ctypes.byref(k.c()), prec, int(n), _ptr(psi0s), _ptr(targets), _ptr(F),
              _ptr(beta), _ptr(beta_cols), _ptr(grad), _ptr(states), int(ckpt_every),
              1 if centred else 0, ws.ptr, ws.nbytes, _stream()]
    if basis is None:
        _lib.check("grape_gradient_columns", lib.grape_gradient_columns(
            ctypes.byref(h.c()), _ptr(u), *common))
    else:
        _lib.check("grape_gradient_columns_pe", lib.grape_gradient_columns_pe(
            ctypes.byref(h.c()), basis.ref(), _ptr(u), *common))
    return ColumnsResult(F=F, beta=beta, beta_cols=beta_cols, grad=grad, states=states)


def grape_ascent_update(u: torch.Tensor, grad: torch.Tensor, eta: float) -> torch.Tensor:
    """u += eta * grad / max|grad| in place, on the device."""
    N = u.numel()
    _f64(u, N, "u")
    _f64(grad, N, "grad")
    _lib.check("grape_ascent_update", _lib.load().grape_ascent_update(
        _ptr(u), _ptr(grad), N, float(eta), _stream()))
    return u


def debug_index_map(L: int, s0: int, count: int, device=None):
    """(n_anti, partner_mask) for s = s0..s0+count-1, computed on the device."""
    dev = device or torch.device("cuda")
    n_anti = torch.empty(count, dtype=torch.int32, device=dev)
    pmask = torch.empty(count, dtype=torch.int32, device=dev)
    _lib.check("kg_debug_index_map", _lib.load().kg_debug_index_map(
        int(L), int(s0), int(count), _ptr(n_anti), _ptr(pmask), _stream()))
    return n_anti, pmask


class profile:
    """Context manager around kg_profile_begin/kg_profile_end (sampled HIP-event
    timing of every kernel class); `.result` maps class -> {launches, ms, bytes}."""

    def __init__(self, sample_every: int = 1, max_launches: int = 1 << 17):
        self.sample_every = sample_every
        self.max_launches = max_launches
        self.result = None

    def __enter__(self):
        _lib.check("kg_profile_begin",
                   _lib.load().kg_profile_begin(self.sample_every, self.max_launches))
        return self

    def __exit__(self, *exc):
        n = len(_lib.PROF_CLASSES)
        launches = (ctypes.c_int64 * n)()
        ms = (ctypes.c_double * n)()
        nbytes = (ctypes.c_double * n)()
        _lib.check("kg_profile_end", _lib.load().kg_profile_end(
            ctypes.cast(launches, ctypes.c_void_p), ctypes.cast(ms, ctypes.c_void_p),
            ctypes.cast(nbytes, ctypes.c_void_p)))
        self.result = {c: {"launches": int(launches[i]), "ms": float(ms[i]),
                           "bytes": float(nbytes[i])}
                       for i, c in enumerate(_lib.PROF_CLASSES)}
        return False
