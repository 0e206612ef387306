"""Host logic of the batched form (no GPU): the Krylov-dimension choice meets its
accuracy target on the oracle, and the team planner respects the grid."""

import numpy as np
import pytest
import scipy.linalg as sla

import workloads
from oracle import krylov, model
from paper_2010_03598_amd import batched


def test_error_bound_decreases_and_choice_meets_target_on_oracle():
    L, J, Delta, dt, N = 10, 1.0, 1.5, 0.05, 300
    m = batched.choose_m(L, J, Delta, 1, 1.0, dt, N)
    assert 8 <= m <= 24
    norm_h = (L - 1) * J * (0.5 + Delta / 4) + 0.5
    b = [batched.lanczos_error_bound(0.5 * norm_h * dt, k) for k in range(6, 25)]
    assert all(x >= y for x, y in zip(b, b[1:]))
    assert batched.lanczos_error_bound(0.5 * norm_h * dt, m) <= 1e-8 / N
    # the oracle's Krylov propagation at the chosen m reaches the target against expm
    rng = np.random.default_rng(0)
    psi = workloads.random_state(rng, 1 << L)
    ch = model.Chain(L, J, Delta, 0, 1)
    H = model.xxz_dense(L, J, Delta) + 1.0 * model.hc_dense(L, 0, 1)
    out = krylov.expv(lambda v: ch.apply(1.0, v), psi, dt, m, True)
    assert np.linalg.norm(out - sla.expm(-1j * dt * H) @ psi) <= 1e-8 / N


def test_choose_m_on_batched_workload():
    ms = [batched.choose_m(c.L, c.J, c.Delta, 1, float(np.abs(c.u).max()), c.dt, c.N)
          for c in workloads.batched()]
    assert min(ms) >= 8 and max(ms) <= 24


class FakeChain:
    def __init__(self, L, N, m):
        self.h = type("H", (), {"L": L})()
        self.N, self.m = N, m


def test_plan_teams_fits_grid_and_balances():
    rng = np.random.default_rng(3)
    chains = [FakeChain(int(rng.integers(10, 17)), int(rng.integers(50, 301)), 12) for _ in range(64)]
    teams = batched.plan_teams(chains, 256)
    assert len(teams) == 64 and sum(teams) <= 256 and min(teams) >= 1
    for c, t in zip(chains, teams):
        assert t <= max(1, (1 << c.h.L) // batched.TILE) and (t & (t - 1)) == 0
    span = max(batched.work(c) / t for c, t in zip(chains, teams))
    naive = max(batched.work(c) for c in chains)
    assert span <= naive
    with pytest.raises(ValueError):
        batched.plan_teams(chains, 10)
