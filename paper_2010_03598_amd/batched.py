"""Batched form: many chains of uneven L, Delta, N in one persistent launch.

* Krylov dimension per chain: the smallest m in [m_min, m_max] for which the
  a-priori error bound of the Lanczos approximation of exp(-itH)v
  (Hochbruck & Lubich, SIAM J. Numer. Anal. 34 (1997), Theorem 2 for a
  skew-Hermitian argument) is below tol / N per slice.  The spectral interval
  of H = H0 + u Hc is bounded by Gershgorin's theorem:
      ||H|| <= (L-1) |J| (1/2 + |Delta|/4) + max|u| * (1/2) * (#control sites).
  This replaces the a-posteriori estimates the paper points to for the choice
  of the Krylov dimension; the bound is pessimistic, so the chosen m is safe.
* Team shapes: the planner gives each chain a team of workgroups, doubling the
  team of the chain with the largest estimated time (work / team) while the
  persistent grid has room; the autotuner times a few plans (different caps on
  the team size) on the GPU and keeps the fastest.
* Packing: controls, states, gradients and scratch of all chains in single
  device buffers, addressed by the kg_chain descriptors.
* Step capture: gradient of every chain plus the per-chain steepest-ascent
  update, captured once in a HIP graph and replayed.
"""

from __future__ import annotations

import ctypes
import dataclasses
import math
import time
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import KG_HC_SX, KgChain
from .api import XXZ, _ptr, _stream, grape_ascent_update

TILE = 1024            # amplitudes per tile of the persistent kernel (one per thread)


def lanczos_error_bound(rho_t: float, m: int) -> float:
    """Hochbruck-Lubich bound for ||exp(tA)v - V exp(tT) e_1|| with A skew-Hermitian,
    spectrum on an imaginary interval of length 4*rho, rho_t = rho*t, m >= 2 rho_t."""
    if m < 2 * rho_t:
        return math.inf
    return 12.0 * math.exp(-(rho_t ** 2) / m) * (math.e * rho_t / m) ** m


def choose_m(L: int, J: float, Delta: float, n_sites: int, umax: float, dt: float, N: int,
             tol: float = 1e-8, m_min: int = 8, m_max: int = 24) -> int:
    norm_h = (L - 1) * abs(J) * (0.5 + abs(Delta) / 4.0) + abs(umax) * 0.5 * n_sites
    rho_t = 0.5 * norm_h * abs(dt)      # spectrum of -i dt H on an interval of length 2 dt ||H||
    for m in range(m_min, m_max + 1):
        if lanczos_error_bound(rho_t, m) <= tol / N:
            return m
    return m_max


@dataclasses.dataclass
class BatchChain:
    h: XXZ
    N: int
    dt: float
    m: int
    u: torch.Tensor          # (N,) float64 (host or device)
    psi0: torch.Tensor       # (2^L,) complex
    target: torch.Tensor
    reorth: bool = True


def work(c: BatchChain) -> float:
    """Vector traffic of one gradient, in amplitude passes: 2N Krylov calls of
    about m^2 + 3m vector passes each over 2^L amplitudes."""
    return 2.0 * c.N * (c.m * c.m + 3 * c.m) * (1 << c.h.L)


def plan_teams(chains: Sequence[BatchChain], n_blocks: int, max_team: int = 64) -> List[int]:
    """Greedy makespan balancing: start with one workgroup per chain and double the
    team of the currently slowest chain while the grid has room."""
    n = len(chains)
    if n > n_blocks:
        raise ValueError(f"{n} chains need at least {n} workgroups, the grid has {n_blocks}")
    team = [1] * n
    used = n
    cap = [min(max_team, max(1, (1 << c.h.L) // TILE)) for c in chains]
    while True:
        order = sorted(range(n), key=lambda i: -work(chains[i]) / team[i])
        grown = False
        for i in order:
            if team[i] * 2 <= cap[i] and used + team[i] <= n_blocks:
                used += team[i]
                team[i] *= 2
                grown = True
            break
        if not grown:
            break
    return team


class Batch:
    """Packed device buffers and descriptors for a set of chains."""

    def __init__(self, chains: Sequence[BatchChain], n_blocks: Optional[int] = None,
                 teams: Optional[Sequence[int]] = None, max_team: int = 64, device=None):
        dev = device or torch.device("cuda")
        self.chains = list(chains)
        if n_blocks is None:
            n_blocks = torch.cuda.get_device_properties(dev).multi_processor_count
        self.n_blocks = int(n_blocks)
        self.teams = list(teams) if teams is not None else plan_teams(self.chains, self.n_blocks,
                                                                       max_team)
        lib = _lib.load()
        descs = (KgChain * len(self.chains))()
        off_u = off_vec = off_states = off_ws = 0
        first = 0
        self.offsets = []
        for i, c in enumerate(self.chains):
            D = 1 << c.h.L
            wsb = int(lib.kg_batched_chain_ws_bytes(c.h.L, c.m, self.teams[i]))
            if wsb == 0:
                raise ValueError(f"chain {i}: unsupported L={c.h.L}, m={c.m} or team {self.teams[i]}")
            d = descs[i]
            d.h = c.h.c()
            d.N, d.m, d.reorth = c.N, c.m, 1 if c.reorth else 0
            d.team_first, d.team_size = first, self.teams[i]
            d.dt, d.breakdown_tol = float(c.dt), 0.0
            d.off_u, d.off_vec, d.off_states, d.off_ws = off_u, off_vec, off_states, off_ws
            self.offsets.append((off_u, off_vec, off_states))
            first += self.teams[i]
            off_u += c.N
            off_vec += D
            off_states += c.N * D
            off_ws += (wsb + 255) // 256 * 256
        self.descs = descs
        self.descs_dev = torch.frombuffer(bytearray(bytes(descs)), dtype=torch.uint8).to(dev)
        self.u = torch.cat([c.u.to(torch.float64).reshape(-1) for c in self.chains]).to(dev)
        self.psi0 = torch.cat([c.psi0.to(torch.complex64).reshape(-1) for c in self.chains]).to(dev)
        self.target = torch.cat([c.target.to(torch.complex64).reshape(-1)
                                 for c in self.chains]).to(dev)
        self.states = torch.empty(off_states, dtype=torch.complex64, device=dev)
        self.grad = torch.zeros(off_u, dtype=torch.float64, device=dev)
        self.F = torch.zeros(len(self.chains), dtype=torch.float64, device=dev)
        self.beta = torch.zeros(2 * len(self.chains), dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws = torch.empty(off_ws + 256, dtype=torch.uint8, device=dev)
        self.ws_off = (-self.ws.data_ptr()) % 256
        self.ws_bytes = off_ws

    def gradient(self) -> None:
        """F and dF/du of every chain (one persistent launch)."""
        _lib.check("grape_gradient_batched", _lib.load().grape_gradient_batched(
            ctypes.cast(self.descs, ctypes.c_void_p), _ptr(self.descs_dev), len(self.chains),
            self.n_blocks, _ptr(self.u), self.u.numel(), _ptr(self.psi0), _ptr(self.target),
            self.psi0.numel(), _ptr(self.states), self.states.numel(), _ptr(self.F), _ptr(self.beta),
            _ptr(self.grad), ctypes.c_void_p(self.ws.data_ptr() + self.ws_off), self.ws_bytes,
            _ptr(self.status), _stream()))

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
             caps: Sequence[int] = (1, 2, 4, 8, 16, 32), reps: int = 1):
    """Time the batched gradient for team-size caps and return (best Batch, timings)."""
    timings = {}
    best = None
    for cap in caps:
        b = Batch(chains, n_blocks=n_blocks, max_team=cap)
        b.gradient()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.gradient()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        b.check_status()
        timings[cap] = {"seconds": t, "teams": list(b.teams)}
        if best is None or t < best[0]:
            best = (t, cap, b)
        else:
            del b
    return best[2], {"best_cap": best[1], "timings": timings}


def from_workload(ws_chains, m: Optional[int] = None, device=None) -> List[BatchChain]:
    """BatchChain list from workloads.Chain records (m from choose_m unless given)."""
    out = []
    for c in ws_chains:
        mm = m if m is not None else choose_m(c.L, c.J, c.Delta, bin(c.hc_sites).count("1"),
                                              float(abs(c.u).max()), c.dt, c.N)
        out.append(BatchChain(h=XXZ(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites), N=c.N, dt=c.dt,
                              m=mm, u=torch.tensor(c.u, dtype=torch.float64),
                              psi0=torch.tensor(c.psi0), target=torch.tensor(c.target)))
    return out


__all__ = ["BatchChain", "Batch", "CapturedStep", "autotune", "choose_m", "plan_teams",
           "lanczos_error_bound", "from_workload", "KG_HC_SX"]
