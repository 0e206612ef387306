"""Batched form: many chains of uneven L, Delta, N in one persistent launch.

The planning lives in the C library (kg_batched_plan, kg_batched_autotune);
this module only packs the chains' data into device buffers and calls it:

* Krylov dimension per chain: the smallest m in [m_min, m_max] whose a-priori
  Lanczos error bound (Hochbruck & Lubich, Theorem 2) is below tol / N per
  slice, with the spectral radius of H0 + u Hc from Gershgorin's theorem.
* Team shapes: one workgroup per chain, then the team of the chain with the
  largest estimated time doubled while the persistent grid has room; the
  autotuner times a few caps on the team size on the GPU and keeps the
  fastest.
* Packing: controls, states, gradients and scratch of all chains in single
  device buffers, addressed by the kg_chain descriptors.
* Step capture: gradient of every chain plus the per-chain steepest-ascent
  update, captured once in a HIP graph and replayed.
"""

from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import KG_HC_SX, KgBatchPlan, KgChain
from .api import XXZ, _ptr, _stream, grape_ascent_update

TOL = 1e-8             # accuracy per sweep of the Krylov-dimension choice
M_MIN, M_MAX = 8, 24   # range of the Krylov-dimension choice


@dataclasses.dataclass
class BatchChain:
    h: XXZ
    N: int
    dt: float
    m: int                   # Krylov dimension; 0: chosen by the planner
    u: torch.Tensor          # (N,) float64 (host or device)
    psi0: torch.Tensor       # (2^L,) complex
    target: torch.Tensor
    reorth: bool = True


def plan(chains: Sequence[BatchChain], n_blocks: int, max_team: int = 64,
         teams: Optional[Sequence[int]] = None):
    """Descriptors and buffer sizes of a batch from kg_batched_plan (host only):
    (kg_chain array, KgBatchPlan)."""
    n = len(chains)
    descs = (KgChain * n)()
    umax = (ctypes.c_double * n)()
    for i, c in enumerate(chains):
        d = descs[i]
        d.h = c.h.c()
        d.N, d.m, d.reorth = int(c.N), int(c.m), 1 if c.reorth else 0
        d.dt, d.breakdown_tol = float(c.dt), 0.0
        d.team_size = int(teams[i]) if teams is not None else 0
        umax[i] = float(torch.as_tensor(c.u).abs().max())
    p = KgBatchPlan()
    _lib.check("kg_batched_plan", _lib.load().kg_batched_plan(
        ctypes.cast(descs, ctypes.c_void_p), n, ctypes.cast(umax, ctypes.c_void_p), int(n_blocks),
        int(max_team), 1 if teams is not None else 0, TOL, M_MIN, M_MAX, ctypes.byref(p)))
    return descs, p


class Batch:
    """Packed device buffers and descriptors for a set of chains."""

    def __init__(self, chains: Sequence[BatchChain], n_blocks: Optional[int] = None,
                 teams: Optional[Sequence[int]] = None, max_team: int = 64, device=None,
                 ws_caps: Sequence[int] = ()):
        """Plan (kg_batched_plan) and allocate; `ws_caps`: further team-size caps whose
        plans the workspace must also hold (for kg_batched_autotune)."""
        dev = device or torch.device("cuda")
        self.chains = list(chains)
        if n_blocks is None:
            n_blocks = torch.cuda.get_device_properties(dev).multi_processor_count
        self.n_blocks = int(n_blocks)
        descs, p = plan(self.chains, self.n_blocks, max_team, teams)
        ws_bytes = int(p.ws_bytes)
        for cap in ws_caps:
            ws_bytes = max(ws_bytes, int(plan(self.chains, self.n_blocks, cap)[1].ws_bytes))
        self.descs = descs
        self.teams = [int(d.team_size) for d in descs]
        self.m = [int(d.m) for d in descs]
        self.offsets = [(int(d.off_u), int(d.off_vec), int(d.off_states)) for d in descs]
        self.descs_dev = torch.frombuffer(bytearray(bytes(descs)), dtype=torch.uint8).to(dev)
        self.u = torch.cat([c.u.to(torch.float64).reshape(-1) for c in self.chains]).to(dev)
        self.psi0 = torch.cat([c.psi0.to(torch.complex64).reshape(-1) for c in self.chains]).to(dev)
        self.target = torch.cat([c.target.to(torch.complex64).reshape(-1)
                                 for c in self.chains]).to(dev)
        assert self.u.numel() == p.u_len and self.psi0.numel() == p.vec_len
        self.states = torch.empty(int(p.states_len), dtype=torch.complex64, device=dev)
        self.grad = torch.zeros(int(p.u_len), dtype=torch.float64, device=dev)
        self.F = torch.zeros(len(self.chains), dtype=torch.float64, device=dev)
        self.beta = torch.zeros(2 * len(self.chains), dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
        self.ws_off = (-self.ws.data_ptr()) % 256
        self.ws_bytes = ws_bytes

    def _buffers(self):
        return [_ptr(self.u), self.u.numel(), _ptr(self.psi0), _ptr(self.target),
                self.psi0.numel(), _ptr(self.states), self.states.numel(), _ptr(self.F),
                _ptr(self.beta), _ptr(self.grad),
                ctypes.c_void_p(self.ws.data_ptr() + self.ws_off), self.ws_bytes, _ptr(self.status)]

    def gradient(self) -> None:
        """F and dF/du of every chain (one persistent launch)."""
        _lib.check("grape_gradient_batched", _lib.load().grape_gradient_batched(
            ctypes.cast(self.descs, ctypes.c_void_p), _ptr(self.descs_dev), len(self.chains),
            self.n_blocks, *self._buffers(), _stream()))

    def ascent_step(self, eta: float) -> None:
        """Gradient of every chain, then u <- u + eta g / max|g| per chain."""
        self.gradient()
        for i, c in enumerate(self.chains):
            o = self.offsets[i][0]
            grape_ascent_update(self.u[o:o + c.N], self.grad[o:o + c.N], eta)

    def grad_of(self, i: int) -> torch.Tensor:
        o = self.offsets[i][0]
        return self.grad[o:o + self.chains[i].N]

    def check_status(self) -> None:
        if int(self.status.item()) != 0:
            raise RuntimeError("a team barrier of the batched kernel timed out; results invalid")


class CapturedStep:
    """The batched ascent step captured in a HIP graph (torch.cuda.CUDAGraph)."""

    def __init__(self, batch: Batch, eta: float):
        self.batch = batch
        self.eta = eta
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            batch.ascent_step(eta)           # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        from ._graph import capture_guard
        self.graph = torch.cuda.CUDAGraph()
        with capture_guard(), torch.cuda.graph(self.graph):
            batch.ascent_step(eta)

    def replay(self) -> None:
        self.graph.replay()


def autotune(chains: Sequence[BatchChain], n_blocks: Optional[int] = None,
             caps: Sequence[int] = (1, 2, 4, 8, 16, 32, 64), reps: int = 1):
    """kg_batched_autotune over team-size caps: returns (Batch planned with the
    fastest cap, {"best_cap", "timings"})."""
    b = Batch(chains, n_blocks=n_blocks, max_team=max(caps), ws_caps=caps)
    caps_arr = (ctypes.c_int32 * len(caps))(*[int(c) for c in caps])
    ms = (ctypes.c_float * len(caps))()
    best = ctypes.c_int32(0)
    _lib.check("kg_batched_autotune", _lib.load().kg_batched_autotune(
        ctypes.cast(b.descs, ctypes.c_void_p), _ptr(b.descs_dev), len(b.chains), b.n_blocks,
        ctypes.cast(caps_arr, ctypes.c_void_p), len(caps), int(reps), *b._buffers(),
        ctypes.cast(ms, ctypes.c_void_p), ctypes.byref(best), _stream()))
    b.teams = [int(d.team_size) for d in b.descs]
    timings = {int(c): {"seconds": float(ms[q]) * 1e-3} for q, c in enumerate(caps)}
    return b, {"best_cap": int(best.value), "timings": timings, "teams": list(b.teams)}


def from_workload(ws_chains, m: Optional[int] = None, device=None) -> List[BatchChain]:
    """BatchChain list from workloads.Chain records (m = 0, chosen by the planner,
    unless given)."""
    out = []
    for c in ws_chains:
        mm = int(m) if m is not None else 0
        out.append(BatchChain(h=XXZ(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites), N=c.N, dt=c.dt,
                              m=mm, u=torch.tensor(c.u, dtype=torch.float64),
                              psi0=torch.tensor(c.psi0), target=torch.tensor(c.target)))
    return out


__all__ = ["BatchChain", "Batch", "CapturedStep", "autotune", "plan", "from_workload", "KG_HC_SX"]
