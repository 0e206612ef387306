"""Pins of oracle.dimension (the Krylov dimension of the batched form): the
Gershgorin norm bounds the spectrum, the Hochbruck-Lubich bound holds for the
oracle's Lanczos propagator against dense exponentials, and the choice is the
smallest dimension that meets its target."""

import numpy as np
import pytest
import scipy.linalg as sla

import workloads
from oracle import dimension, krylov, model


@pytest.mark.parametrize("L,J,Delta,kind,sites", [(6, 1.0, 0.5, 0, 1), (8, -0.7, 1.5, 0, 1 << 3),
                                                  (7, 1.3, 0.0, 1, 0b1000001), (9, 1.0, 1.0, 1, 1)])
@pytest.mark.parametrize("u", [0.0, 1.0, -2.0])
def test_gershgorin_bounds_the_spectrum(L, J, Delta, kind, sites, u):
    H = model.xxz_dense(L, J, Delta) + u * model.hc_dense(L, kind, sites)
    rho = np.abs(np.linalg.eigvalsh(H)).max()
    g = dimension.gershgorin_norm(L, J, Delta, bin(sites).count("1"), abs(u))
    assert rho <= g * (1 + 1e-14)
    # tight for the chain's own maximal row sum in the S^x-free XX case
    if kind == 0 and u == 0.0 and Delta == 0.0:
        assert g <= 1.1 * (L - 1) * abs(J) / 2 + 1e-12


@pytest.mark.parametrize("dt,m", [(0.05, 4), (0.1, 6), (0.3, 8), (0.5, 10), (0.2, 5)])
def test_bound_holds_for_lanczos(dt, m):
    L, J, Delta = 8, 1.0, 1.2
    rng = np.random.default_rng(m)
    ch = model.Chain(L, J, Delta, 0, 1)
    u = 0.8
    H = model.xxz_dense(L, J, Delta) + u * model.hc_dense(L, 0, 1)
    rho = 0.5 * dt * dimension.gershgorin_norm(L, J, Delta, 1, u)
    bound = dimension.hochbruck_lubich(rho, m)
    for _ in range(4):
        psi = workloads.random_state(rng, 1 << L)
        out = krylov.expv(lambda v: ch.apply(u, v), psi, dt, m, True)
        err = np.linalg.norm(out - sla.expm(-1j * dt * H) @ psi)
        assert err <= bound


def test_bound_decreases_in_m_past_two_rho():
    rho = 1.7
    b = [dimension.hochbruck_lubich(rho, m) for m in range(4, 30)]
    assert all(x >= y for x, y in zip(b, b[1:]))
    assert dimension.hochbruck_lubich(rho, 3) == np.inf


def test_choice_is_smallest_meeting_the_target():
    for c in workloads.batched()[:20]:
        n = bin(c.hc_sites).count("1")
        um = float(np.abs(c.u).max())
        m = dimension.krylov_dimension(c.L, c.J, c.Delta, n, um, c.dt, c.N)
        rho = 0.5 * c.dt * dimension.gershgorin_norm(c.L, c.J, c.Delta, n, um)
        assert 8 <= m <= 24
        assert dimension.hochbruck_lubich(rho, m) <= 1e-8 / c.N or m == 24
        if m > 8:
            assert dimension.hochbruck_lubich(rho, m - 1) > 1e-8 / c.N


def test_choice_meets_its_target_on_the_oracle():
    L, J, Delta, dt, N = 10, 1.0, 1.5, 0.05, 300
    m = dimension.krylov_dimension(L, J, Delta, 1, 1.0, dt, N)
    rng = np.random.default_rng(0)
    psi = workloads.random_state(rng, 1 << L)
    ch = model.Chain(L, J, Delta, 0, 1)
    H = model.xxz_dense(L, J, Delta) + 1.0 * model.hc_dense(L, 0, 1)
    out = krylov.expv(lambda v: ch.apply(1.0, v), psi, dt, m, True)
    assert np.linalg.norm(out - sla.expm(-1j * dt * H) @ psi) <= 1e-8 / N
