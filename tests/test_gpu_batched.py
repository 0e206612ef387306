"""Batched form on the GPU: one persistent launch for many chains, against the
oracle; determinism; the captured HIP-graph step replayed against eager runs."""

import json
import os

import numpy as np
import pytest
import torch

import paper_2010_03598_amd as kg
import workloads
from oracle import grape, krylov, model
from paper_2010_03598_amd import batched
from tests.gpu_util import host, rel_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def small_chains(n=5, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        L = int(rng.integers(10, 13))
        N = int(rng.integers(8, 25))
        u = rng.uniform(-1, 1, N)
        out.append(workloads.Chain(L=L, J=1.0, Delta=float(rng.uniform(0, 1.5)), hc_kind=0,
                                   hc_sites=1 << int(rng.integers(0, L)), N=N, dt=0.05, m=12,
                                   u=u, psi0=workloads.random_phase_state(rng, 1 << L),
                                   target=workloads.random_phase_state(rng, 1 << L)))
    return out


def oracle_of(c):
    ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    return grape.gradient(ch, c.u, c.psi0, c.target, c.dt, c.m, True,
                          krylov.default_tol(krylov.EPS_C64))


# [3, 5, 2, 3, 3]: teams of any size (the planner's sizes need not be powers of
# two), members holding unequal numbers of tiles, and members holding none
# (chains of 1, 2 or 4 tiles of 2^10 amplitudes)
@pytest.mark.parametrize("teams", [None, [1, 1, 1, 1, 1], [1, 2, 1, 2, 4], [3, 5, 2, 3, 3]])
def test_small_batch_vs_oracle(teams):
    ws = small_chains()
    b = batched.Batch(batched.from_workload(ws, m=12), n_blocks=16, teams=teams)
    b.gradient()
    torch.cuda.synchronize()
    b.check_status()
    F = host(b.F)
    for i, c in enumerate(ws):
        ref = oracle_of(c)
        assert abs(F[i] - ref.F) / ref.F <= 1e-4, i
        assert rel_err(host(b.grad_of(i)), ref.grad) <= 1e-4, i


def test_batched_matches_single_chain_path():
    """Same chains through grape_gradient one by one (complex64): equal to rounding."""
    ws = small_chains(3, seed=5)
    b = batched.Batch(batched.from_workload(ws, m=12), n_blocks=8)
    b.gradient()
    for i, c in enumerate(ws):
        h = kg.XXZ(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
        r = kg.grape_gradient(h, torch.tensor(c.u, device="cuda"), c.dt, kg.Krylov(12),
                              torch.tensor(c.psi0, dtype=torch.complex64, device="cuda"),
                              torch.tensor(c.target, dtype=torch.complex64, device="cuda"))
        assert rel_err(host(b.grad_of(i)), host(r.grad)) <= 1e-5
        assert abs(float(host(b.F)[i]) - float(host(r.F))) / float(host(r.F)) <= 1e-5


def test_deterministic_and_graph_replay():
    ws = small_chains(4, seed=2)
    chains = batched.from_workload(ws, m=12)
    b1 = batched.Batch(chains, n_blocks=12)
    b1.gradient()
    g_first = host(b1.grad).copy()
    b1.gradient()
    assert np.array_equal(host(b1.grad), g_first)
    # eager ascent trajectory
    eager = batched.Batch(chains, n_blocks=12, teams=b1.teams)
    traj = []
    for _ in range(3):
        eager.ascent_step(0.1)
        traj.append((host(eager.F).copy(), host(eager.u).copy()))
    # captured step, replayed; eager work and synchronisation between replays
    cap = batched.Batch(chains, n_blocks=12, teams=b1.teams)
    step = batched.CapturedStep(cap, 0.1)      # the warm-up inside runs step 1 eagerly
    assert np.array_equal(host(cap.u), traj[0][1])
    for r in range(1, 3):
        _ = torch.randn(1000, device="cuda").sum()       # unrelated eager work
        torch.cuda.synchronize()
        step.replay()
        torch.cuda.synchronize()
        cap.check_status()
        assert np.array_equal(host(cap.F), traj[r][0]), r
        assert np.array_equal(host(cap.u), traj[r][1]), r


def test_full_batched_workload_vs_oracle():
    """64 chains, L in 10..16, N in 50..300, one persistent launch (m fixed at the
    oracle's value), against the oracle's stored results."""
    with open(os.path.join(GOLDEN, "batched.json")) as fh:
        gold = json.load(fh)
    ws = workloads.batched()
    b = batched.Batch(batched.from_workload(ws, m=gold["m"]))
    b.gradient()
    torch.cuda.synchronize()
    b.check_status()
    F = host(b.F)
    for i, rec in enumerate(gold["chains"]):
        assert abs(F[i] - rec["F"]) / rec["F"] <= 1e-4, i
        assert rel_err(host(b.grad_of(i)), np.array(rec["grad"])) <= 1e-4, i


def test_autotuned_planned_workload_vs_oracle():
    """The 64-chain workload as the bench times it: Krylov dimensions chosen by the
    C planner, team shapes by the C autotuner; against the oracle run with the
    same dimensions (tests/golden/batched_planned.json)."""
    with open(os.path.join(GOLDEN, "batched_planned.json")) as fh:
        gold = json.load(fh)
    ws = workloads.batched()
    b, info = batched.autotune(batched.from_workload(ws), caps=(2, 8, 32))
    assert b.m == [rec["chain"]["m"] for rec in gold["chains"]]
    assert info["best_cap"] in (2, 8, 32) and sum(b.teams) <= b.n_blocks
    b.gradient()
    torch.cuda.synchronize()
    b.check_status()
    F = host(b.F)
    for i, rec in enumerate(gold["chains"]):
        assert abs(F[i] - rec["F"]) / rec["F"] <= 1e-4, i
        assert rel_err(host(b.grad_of(i)), np.array(rec["grad"])) <= 1e-4, i


def test_autotuned_batch_runs():
    ws = workloads.batched()[:16]
    chains = batched.from_workload(ws)
    best, info = batched.autotune(chains, caps=(1, 4, 16))
    assert info["best_cap"] in (1, 4, 16)
    best.check_status()
    assert np.all(np.isfinite(host(best.grad)))
