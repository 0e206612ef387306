"""krylov_expv on the GPU against the oracle's Lanczos propagator."""

import numpy as np
import pytest
import scipy.linalg as sla
import torch

import paper_2010_03598_amd as kg
import workloads
from oracle import krylov, model
from oracle.model import HC_SX, HC_SZ
from tests.gpu_util import C64, C128, dev_vec, host, tile_bits

pytestmark = pytest.mark.gpu


def oracle_expv(L, J, Delta, kind, sites, u, psi, t, m, reorth, vec_eps=krylov.EPS_C128):
    ch = model.Chain(L, J, Delta, kind, sites)
    return krylov.expv(lambda v: ch.apply(u, v), psi, t, m, reorth, krylov.default_tol(vec_eps),
                       return_info=True)


def gpu_expv(L, J, Delta, kind, sites, u, psi, t, m, reorth, dtype=C128, inplace=False):
    h = kg.XXZ(L, J, Delta, kind, sites)
    v = dev_vec(psi, dtype)
    m_eff = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = kg.krylov_expv(h, u, t, v, kg.Krylov(m, reorth), out=v if inplace else None, m_eff=m_eff)
    return host(out), int(host(m_eff)[0])


@pytest.mark.parametrize("L,m,t,u", [(2, 4, 0.7, 0.2), (3, 5, -0.4, 0.0), (6, 1, 0.05, 0.3),
                                     (6, 2, 0.05, 0.3), (8, 10, 0.1, -0.9), (10, 16, 0.25, 1.7),
                                     (12, 24, 0.5, 0.4), (13, 20, -0.05, -1.0), (16, 16, 0.05, 2.0)])
@pytest.mark.parametrize("reorth", [True, False])
def test_matches_oracle_c128(L, m, t, u, reorth):
    rng = np.random.default_rng(L * 31 + m)
    psi = workloads.random_state(rng, 1 << L)
    ref, lz = oracle_expv(L, 1.0, 0.5, HC_SX, 1, u, psi, t, m, reorth)
    out, m_eff = gpu_expv(L, 1.0, 0.5, HC_SX, 1, u, psi, t, m, reorth)
    assert m_eff == lz.m_eff
    assert np.linalg.norm(out - ref) <= 1e-12


@pytest.mark.parametrize("L,m", [(8, 10), (14, 20), (17, 24)])
def test_matches_oracle_c64(L, m):
    rng = np.random.default_rng(L)
    psi = workloads.random_state(rng, 1 << L)
    ref, _ = oracle_expv(L, 1.0, 1.0, HC_SX, 1, 0.6, psi, 0.05, m, True)
    out, _ = gpu_expv(L, 1.0, 1.0, HC_SX, 1, 0.6, psi, 0.05, m, True, dtype=C64)
    assert np.linalg.norm(out - ref) <= 1e-5


@pytest.mark.parametrize("L,m", [(12, 32), (13, 40), (14, 48), (12, 64), (14, 64)])
@pytest.mark.parametrize("reorth", [True, False])
@pytest.mark.parametrize("dtype,tol", [(C128, 1e-12), (C64, 1e-5)])
def test_large_krylov_dimension(L, m, reorth, dtype, tol):
    """Krylov dimensions up to the largest the library accepts (64: a projection
    window of one vector per lane, every column of the reduction rows in use)."""
    rng = np.random.default_rng(L * 97 + m)
    psi = workloads.random_state(rng, 1 << L)
    eps = krylov.EPS_C128 if dtype == C128 else krylov.EPS_C64
    ref, lz = oracle_expv(L, 1.0, 0.8, HC_SX, 1, -0.45, psi, 0.6, m, reorth, eps)
    out, m_eff = gpu_expv(L, 1.0, 0.8, HC_SX, 1, -0.45, psi, 0.6, m, reorth, dtype=dtype)
    assert m_eff == lz.m_eff == m
    assert np.linalg.norm(out - ref) <= tol


@pytest.mark.parametrize("tb", [6, 7, 8, 9, 10, 11, 12])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_every_tiling(tb, dtype):
    L, m = 14, 12
    rng = np.random.default_rng(tb + 50)
    psi = workloads.random_state(rng, 1 << L)
    ref, _ = oracle_expv(L, 1.0, 0.5, HC_SZ, 0b1001 << 4, -0.7, psi, 0.2, m, True)
    with tile_bits(tb):
        out, m_eff = gpu_expv(L, 1.0, 0.5, HC_SZ, 0b1001 << 4, -0.7, psi, 0.2, m, True, dtype=dtype)
    assert m_eff == m
    assert np.linalg.norm(out - ref) <= (1e-12 if dtype == C128 else 1e-5)


def test_in_place_and_norm_scaling():
    L = 11
    rng = np.random.default_rng(2)
    psi = 0.3 * workloads.random_state(rng, 1 << L)
    ref, _ = oracle_expv(L, 1.0, 0.5, HC_SX, 1, 0.1, psi, 0.3, 14, True)
    out, _ = gpu_expv(L, 1.0, 0.5, HC_SX, 1, 0.1, psi, 0.3, 14, True, inplace=True)
    assert np.linalg.norm(out - ref) <= 1e-12
    assert abs(np.linalg.norm(out) - 0.3) <= 1e-12


def test_unitarity_and_reversibility():
    L = 16
    rng = np.random.default_rng(16)
    psi = workloads.random_phase_state(rng, 1 << L)
    h = kg.XXZ(L, 1.0, 1.0)
    v = dev_vec(psi)
    k = kg.Krylov(20)
    out = kg.krylov_expv(h, 0.8, 0.05, v, k)
    back = kg.krylov_expv(h, 0.8, -0.05, out, k)
    assert abs(np.linalg.norm(host(out)) - 1.0) <= 1e-12
    assert np.linalg.norm(host(back) - psi) <= 1e-12


@pytest.mark.parametrize("dtype", [C128, C64])
def test_breakdown_and_sector_leakage(dtype):
    """S^z control keeps the one-magnon sector invariant: the basis closes at m_eff = L
    and amplitudes outside the sector stay exactly zero."""
    L = 8
    psi = workloads.basis_state(L, workloads.basis_index("u" + "d" * 7))
    sites = 1 | (1 << 7)
    out, m_eff = gpu_expv(L, 1.0, 0.5, HC_SZ, sites, 0.6, psi, 0.5, 12, True, dtype=dtype)
    tol_vec = krylov.EPS_C128 if dtype == C128 else krylov.EPS_C64
    _, lz = oracle_expv(L, 1.0, 0.5, HC_SZ, sites, 0.6, psi, 0.5, 12, True, tol_vec)
    assert m_eff == lz.m_eff == 8
    sector = np.array([bin(s).count("1") == L - 1 for s in range(1 << L)])
    assert np.all(out[~sector] == 0)
    H = model.xxz_dense(L, 1.0, 0.5) + 0.6 * model.hc_dense(L, HC_SZ, sites)
    ref = sla.expm(-0.5j * H) @ psi
    assert np.linalg.norm(out - ref) <= (1e-12 if dtype == C128 else 1e-5)


def test_eigenstate_breaks_down_at_one():
    L = 9
    psi = workloads.basis_state(L, 0)     # all up: eigenstate of H0 and of S^z controls
    out, m_eff = gpu_expv(L, 1.0, 0.5, HC_SZ, 1, 0.25, psi, 0.8, 10, True)
    assert m_eff == 1
    E = 0.25 * 1.0 * 0.5 * (L - 1) + 0.25 * 0.5
    assert abs(out[0] - np.exp(-0.8j * E)) < 1e-14
    assert np.count_nonzero(out) == 1


def test_zero_input():
    L = 7
    out, m_eff = gpu_expv(L, 1.0, 0.5, HC_SX, 1, 0.1, np.zeros(1 << L), 0.2, 6, True)
    assert m_eff == 0 and np.all(out == 0)


def test_single_magnon_closed_form_large():
    """XX chain at L=20: one up spin spreading from site 1 (textbook hopping amplitudes)."""
    L, t = 20, 0.4
    psi = workloads.basis_state(L, workloads.basis_index("u" + "d" * (L - 1)))
    out, _ = gpu_expv(L, 1.0, 0.0, HC_SX, 1, 0.0, psi, t, 24, True)
    k = np.arange(1, L + 1)
    for n in range(1, L + 1):
        amp = np.sum(2.0 / (L + 1) * np.sin(np.pi * k / (L + 1)) * np.sin(np.pi * k * n / (L + 1))
                     * np.exp(-1j * np.cos(np.pi * k / (L + 1)) * t))
        idx = workloads.basis_index("d" * (n - 1) + "u" + "d" * (L - n))
        assert abs(out[idx] - amp) < 1e-12


def test_deterministic():
    L = 18
    rng = np.random.default_rng(18)
    psi = workloads.random_phase_state(rng, 1 << L)
    a, _ = gpu_expv(L, 1.0, 0.5, HC_SX, 1, 0.3, psi, 0.05, 20, True, dtype=C64)
    b, _ = gpu_expv(L, 1.0, 0.5, HC_SX, 1, 0.3, psi, 0.05, 20, True, dtype=C64)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("u,t", [(1e12, 0.1), (0.3, 1e9)])
@pytest.mark.parametrize("dtype", [C64, C128])
def test_exponential_out_of_range_gives_nan(u, t, dtype):
    """|t| ||T|| beyond the evaluated range ends the call with a NaN output
    instead of an unbounded number of Taylor sub-steps."""
    rng = np.random.default_rng(4)
    psi = workloads.random_state(rng, 1 << 8)
    out, _ = gpu_expv(8, 1.0, 0.5, HC_SX, 1, u, psi, t, 8, True, dtype=dtype)
    assert np.isnan(out).all()


def test_non_finite_amplitude_by_value_is_rejected():
    psi = workloads.random_state(np.random.default_rng(4), 1 << 8)
    with pytest.raises(kg.KgError):
        gpu_expv(8, 1.0, 0.5, HC_SX, 1, float("inf"), psi, 0.1, 8, True)


@pytest.mark.parametrize("dtype", [C64, C128])
def test_non_finite_amplitude_on_the_device_gives_nan(dtype):
    """A non-finite control amplitude in device memory (not checked on the
    host) makes the fidelity NaN; the sweep still ends."""
    rng = np.random.default_rng(5)
    psi0 = dev_vec(workloads.random_state(rng, 1 << 8), dtype)
    f = dev_vec(workloads.random_state(rng, 1 << 8), dtype)
    u = torch.tensor([0.2, float("inf"), -0.1], dtype=torch.float64, device="cuda")
    r = kg.grape_forward(kg.XXZ(8, 1.0, 0.5), u, 0.1, kg.Krylov(8), psi0, f)
    assert np.isnan(float(host(r.F)))


@pytest.mark.parametrize("dtype", [C64, C128])
def test_non_finite_input_gives_nan(dtype):
    psi = workloads.random_state(np.random.default_rng(6), 1 << 8)
    psi[3] = np.nan
    out, m_eff = gpu_expv(8, 1.0, 0.5, HC_SX, 1, 0.3, psi, 0.1, 8, True, dtype=dtype)
    assert np.isnan(out).all() and m_eff == 1
