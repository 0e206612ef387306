"""Host logic of the batched form (no GPU): kg_batched_plan through the C ABI.
Its Krylov dimensions equal the oracle's choice chain by chain (bit-exact
integers), the stored batched golden was computed with those dimensions, and the
team planner respects the grid, the caps and the packing."""

import ctypes
import json
import os

import numpy as np
import pytest

import workloads
from oracle import dimension
from paper_2010_03598_amd import _lib
from paper_2010_03598_amd._lib import KgBatchPlan, KgChain, KgXxz

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TILE = 1024


def c_plan(chains, n_blocks, max_team=64, teams=None, tol=1e-8, m_min=8, m_max=24, ms=None):
    n = len(chains)
    descs = (KgChain * n)()
    umax = (ctypes.c_double * n)()
    for i, c in enumerate(chains):
        d = descs[i]
        d.h = KgXxz(c.L, c.hc_kind, c.J, c.Delta, c.hc_sites)
        d.N, d.m, d.reorth, d.dt = c.N, 0 if ms is None else ms[i], 1, c.dt
        d.team_size = 0 if teams is None else teams[i]
        umax[i] = float(np.abs(c.u).max())
    p = KgBatchPlan()
    st = _lib.load().kg_batched_plan(ctypes.cast(descs, ctypes.c_void_p), n,
                                     ctypes.cast(umax, ctypes.c_void_p), n_blocks, max_team,
                                     0 if teams is None else 1, tol, m_min, m_max,
                                     ctypes.byref(p))
    return st, descs, p


def oracle_m(c, tol=1e-8):
    return dimension.krylov_dimension(c.L, c.J, c.Delta, bin(c.hc_sites).count("1"),
                                      float(np.abs(c.u).max()), c.dt, c.N, tol)


def test_dimensions_equal_the_oracle_choice():
    chains = workloads.batched()
    st, descs, _ = c_plan(chains, 256)
    assert st == _lib.KG_OK, _lib.last_error()
    assert [d.m for d in descs] == [oracle_m(c) for c in chains]
    # a tighter and a looser accuracy move the choice the same way on both sides
    for tol in (1e-12, 1e-4):
        st, descs, _ = c_plan(chains[:16], 256, tol=tol)
        assert [d.m for d in descs] == [oracle_m(c, tol) for c in chains[:16]]


def test_golden_batch_was_computed_with_the_planned_dimensions():
    with open(os.path.join(GOLDEN, "batched_planned.json")) as fh:
        gold = json.load(fh)
    _, descs, _ = c_plan(workloads.batched(), 256)
    assert [d.m for d in descs] == [rec["chain"]["m"] for rec in gold["chains"]]


def modelled_time(c, m, team):
    """The planner's step model: per Lanczos step 5 us fixed plus 0.65 us per
    tile of the busiest member and window vector ((m + 6) / 2 on average)."""
    tiles = max(1, (1 << c.L) // TILE)
    per = -(-tiles // team)
    return 2.0 * c.N * m * (5.0 + 0.65 * 0.5 * (m + 6) * per)


@pytest.mark.parametrize("n_blocks,max_team", [(256, 64), (128, 8), (64, 1), (300, 16), (256, 32)])
def test_teams_fit_grid_caps_and_balance(n_blocks, max_team):
    chains = workloads.batched()
    st, descs, p = c_plan(chains, n_blocks, max_team)
    assert st == _lib.KG_OK, _lib.last_error()
    teams = [d.team_size for d in descs]
    assert sum(teams) == p.blocks_used <= n_blocks and min(teams) >= 1
    caps = [min(max_team, max(1, (1 << c.L) // TILE)) for c in chains]
    assert all(t <= cap for t, cap in zip(teams, caps))
    # no team is larger than the smallest one holding the same tiles per member
    for c, t in zip(chains, teams):
        tiles = max(1, (1 << c.L) // TILE)
        assert t == 1 or -(-tiles // (t - 1)) > -(-tiles // t)
    # the greedy stops at the chain with the largest modelled time: it holds one
    # tile per member, or the next team that would hold fewer exceeds its cap or
    # the grid
    span = [modelled_time(c, d.m, d.team_size) for c, d in zip(chains, descs)]
    i = int(np.argmax(span))
    tiles = max(1, (1 << chains[i].L) // TILE)
    per = -(-tiles // teams[i])
    if per > 1:
        nxt = -(-tiles // (per - 1))
        assert nxt > caps[i] or p.blocks_used + nxt - teams[i] > n_blocks
    # one workgroup per chain is never better
    assert max(span) <= max(modelled_time(c, d.m, 1) for c, d in zip(chains, descs))


def test_planned_makespan_beats_power_of_two_teams():
    """On the 64-chain workload the modelled slowest chain is faster than with
    teams restricted to powers of two by doubling (the earlier planner)."""
    chains = workloads.batched()
    st, descs, p = c_plan(chains, 256, 64)
    assert st == _lib.KG_OK
    ms = [d.m for d in descs]
    planned = max(modelled_time(c, m, d.team_size) for c, m, d in zip(chains, ms, descs))
    teams = [1] * len(chains)
    used = len(chains)
    work = [2.0 * c.N * (m * m + 3 * m) * (1 << c.L) for c, m in zip(chains, ms)]
    while True:
        i = max(range(len(chains)), key=lambda j: (work[j] / teams[j], -j))
        cap = min(64, max(1, (1 << chains[i].L) // TILE))
        if teams[i] * 2 > cap or used + teams[i] > 256:
            break
        used += teams[i]
        teams[i] *= 2
    doubling = max(modelled_time(c, m, t) for c, m, t in zip(chains, ms, teams))
    assert planned < 0.9 * doubling


def test_packing_is_contiguous():
    chains = workloads.batched()[:9]
    st, descs, p = c_plan(chains, 64)
    assert st == _lib.KG_OK
    off_u = off_vec = off_states = off_ws = first = 0
    for c, d in zip(chains, descs):
        assert (d.off_u, d.off_vec, d.off_states, d.off_ws, d.team_first) == \
               (off_u, off_vec, off_states, off_ws, first)
        assert d.off_ws % 256 == 0
        wsb = _lib.load().kg_batched_chain_ws_bytes(c.L, d.m, d.team_size)
        off_u += c.N
        off_vec += 1 << c.L
        off_states += c.N << c.L
        off_ws += (wsb + 255) // 256 * 256
        first += d.team_size
    assert (p.u_len, p.vec_len, p.states_len, p.ws_bytes) == (off_u, off_vec, off_states, off_ws)


def test_kept_teams_and_given_dimensions():
    chains = workloads.batched()[:5]
    st, descs, p = c_plan(chains, 32, teams=[1, 2, 4, 1, 2], ms=[9, 10, 11, 12, 13])
    assert st == _lib.KG_OK
    assert [d.team_size for d in descs] == [1, 2, 4, 1, 2]
    assert [d.m for d in descs] == [9, 10, 11, 12, 13]
    assert [d.team_first for d in descs] == [0, 1, 3, 7, 8]


@pytest.mark.parametrize("kw", [dict(n_blocks=3), dict(n_blocks=64, max_team=0),
                                dict(n_blocks=64, max_team=65), dict(n_blocks=64, tol=0.0),
                                dict(n_blocks=64, m_min=10, m_max=9)])
def test_invalid_arguments(kw):
    chains = workloads.batched()[:5]
    st, _, _ = c_plan(chains, **kw)
    assert st == _lib.KG_EINVAL and _lib.last_error()


def test_grid_too_small_for_kept_teams():
    chains = workloads.batched()[:3]
    st, _, _ = c_plan(chains, 4, teams=[2, 2, 2])
    assert st == _lib.KG_EINVAL
