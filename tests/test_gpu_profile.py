"""Sampled kernel timing (kg_profile_begin/end): every launch of a gradient
sampled, the records counted per kernel class, the durations taken by the
dispatch itself (they add up to less than the wall time of the gradient),
and the algorithmic bytes filed per class as the passes define them."""

import time

import numpy as np
import pytest
import torch

import paper_2010_03598_amd as kg
import workloads
from tests.gpu_util import C64, dev_vec

pytestmark = pytest.mark.gpu


def test_every_launch_sampled_once():
    L, N, m = 14, 6, 10
    c = workloads._random_chain(21, L=L, Delta=0.8, N=N, dt=0.05, m=m, urange=1.0)
    h = kg.XXZ(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    u = torch.tensor(c.u, dtype=torch.float64, device="cuda")
    psi0, f = dev_vec(c.psi0, C64), dev_vec(c.target, C64)
    k = kg.Krylov(m)
    ws = kg.Workspace(h, k, C64)
    kg.grape_gradient(h, u, c.dt, k, psi0, f, workspace=ws)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with kg.profile(sample_every=1) as p:
        kg.grape_gradient(h, u, c.dt, k, psi0, f, workspace=ws)
        torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    r = p.result
    calls = 2 * N - 1                      # store-all: N forward, N - 1 costate calls
    assert r["pass_a"]["launches"] == calls * m
    assert r["pass_b"]["launches"] == calls * (m - 1)
    assert r["combine"]["launches"] == calls
    assert r["bracket"]["launches"] == N
    assert r["overlap"]["launches"] == 1
    V = 8 << L
    # pass A: v_k read and y written (the last step only reads); pass B: y,
    # the window (all earlier vectors) and the new vector; combination m + 1
    assert r["pass_a"]["bytes"] == calls * V * (2 * (m - 1) + 1)
    assert r["pass_b"]["bytes"] == calls * V * sum(k + 1 + 2 for k in range(m - 1))
    assert r["combine"]["bytes"] == calls * V * (m + 1)
    total = sum(v["ms"] for v in r.values())
    assert all(v["ms"] > 0 for v in r.values() if v["launches"])
    assert total < wall_ms
