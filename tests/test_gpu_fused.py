"""The one-block Krylov call (the whole Lanczos recurrence, the small
exponential and the combination in one launch, with the stored basis in LDS)
used for vectors whose m D amplitudes fit the LDS budget: against the
oracle's Lanczos propagator (App. A, Algorithm 2), the full-space and the
reduced-basis Hamiltonian, breakdowns, degenerate inputs, and against the
tiled multi-launch passes on the same inputs."""

import numpy as np
import pytest
import torch

import paper_2010_03598_amd as kg
import workloads
from oracle import grape, krylov, model, pe
from oracle.model import HC_SX, HC_SZ
from paper_2010_03598_amd import _lib
from tests.gpu_util import C64, C128, dev_vec, host, rel_err, tiled_only

pytestmark = pytest.mark.gpu

# stored basis bytes of the one-block form, as the library's LDS budget
FUSED_LDS = 120 << 10
FUSED_MAX_D = 1024


def fits(D, m, dtype):
    return D <= FUSED_MAX_D and m * D * (16 if dtype == C128 else 8) <= FUSED_LDS


def oracle_expv(L, Delta, kind, sites, u, psi, t, m, reorth, eps):
    ch = model.Chain(L, 1.0, Delta, kind, sites)
    return krylov.expv(lambda v: ch.apply(u, v), psi, t, m, reorth, krylov.default_tol(eps),
                       return_info=True)


def gpu_expv(L, Delta, kind, sites, u, psi, t, m, reorth, dtype):
    h = kg.XXZ(L, 1.0, Delta, kind, sites)
    m_eff = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = kg.krylov_expv(h, u, t, dev_vec(psi, dtype), kg.Krylov(m, reorth), m_eff=m_eff)
    return host(out), int(host(m_eff)[0])


CASES = [(2, 4, HC_SX, 1), (3, 6, HC_SZ, 0b101), (5, 12, HC_SX, 1 << 2), (6, 64, HC_SX, 1),
         (8, 20, HC_SZ, 0b10000001), (8, 30, HC_SX, 1 << 7), (9, 15, HC_SX, 1), (10, 7, HC_SX, 1)]


@pytest.mark.parametrize("L,m,kind,sites", CASES)
@pytest.mark.parametrize("reorth", [True, False])
@pytest.mark.parametrize("dtype,tol", [(C128, 1e-12), (C64, 1e-5)])
def test_matches_oracle(L, m, kind, sites, reorth, dtype, tol):
    assert fits(1 << L, m, dtype)
    rng = np.random.default_rng(L * 13 + m)
    psi = workloads.random_state(rng, 1 << L)
    eps = krylov.EPS_C128 if dtype == C128 else krylov.EPS_C64
    ref, lz = oracle_expv(L, 0.7, kind, sites, -0.55, psi, 0.35, m, reorth, eps)
    out, m_eff = gpu_expv(L, 0.7, kind, sites, -0.55, psi, 0.35, m, reorth, dtype)
    assert m_eff == lz.m_eff
    assert np.linalg.norm(out - ref) <= tol


@pytest.mark.parametrize("L,m", [(6, 10), (8, 20), (9, 15)])
@pytest.mark.parametrize("dtype,tol", [(C128, 1e-13), (C64, 2e-6)])
def test_same_as_tiled_passes(L, m, dtype, tol):
    """Both forms of the Krylov call on the same input agree to rounding, and
    they are different code (their complex64 results differ in the last bits)."""
    rng = np.random.default_rng(L + 500)
    psi = workloads.random_state(rng, 1 << L)
    a, ma = gpu_expv(L, 1.0, HC_SX, 1, 0.8, psi, 0.2, m, True, dtype)
    with tiled_only():
        b, mb = gpu_expv(L, 1.0, HC_SX, 1, 0.8, psi, 0.2, m, True, dtype)
    assert ma == mb == m
    assert np.linalg.norm(a - b) <= tol
    if dtype == C64:
        assert not np.array_equal(a, b)


@pytest.mark.parametrize("dtype", [C128, C64])
def test_breakdown_inside_the_one_magnon_sector(dtype):
    """A single magnon of the open XX chain (Delta = 0, S^z control on both
    ends) stays in the L-dimensional one-magnon sector, and a magnon on the
    middle site stays in its mirror-even part: the basis breaks down before m,
    at the same m_eff as the oracle's."""
    L, m = 7, 12
    psi = np.zeros(1 << L, dtype=np.complex128)
    psi[1 << 3] = 1.0
    eps = krylov.EPS_C128 if dtype == C128 else krylov.EPS_C64
    ref, lz = oracle_expv(L, 0.0, HC_SZ, 0b1000001, 0.3, psi, 0.4, m, True, eps)
    out, m_eff = gpu_expv(L, 0.0, HC_SZ, 0b1000001, 0.3, psi, 0.4, m, True, dtype)
    assert m_eff == lz.m_eff <= L < m
    assert np.linalg.norm(out - ref) <= (1e-12 if dtype == C128 else 1e-5)


def test_eigenstate_and_degenerate_inputs():
    L = 6
    # the all-up state is an eigenstate of the XXZ chain with an S^z control
    psi = np.zeros(1 << L, dtype=np.complex128)
    psi[0] = 2.0
    out, m_eff = gpu_expv(L, 0.5, HC_SZ, 1, 0.4, psi, 0.3, 8, True, C128)
    ref, lz = oracle_expv(L, 0.5, HC_SZ, 1, 0.4, psi, 0.3, 8, True, krylov.EPS_C128)
    assert m_eff == lz.m_eff == 1
    assert np.linalg.norm(out - ref) <= 1e-13
    zero = np.zeros(1 << L, dtype=np.complex128)
    out, m_eff = gpu_expv(L, 0.5, HC_SX, 1, 0.4, zero, 0.3, 8, True, C128)
    assert m_eff == 0 and not out.any()
    bad = workloads.random_state(np.random.default_rng(3), 1 << L)
    bad[5] = np.nan
    for dtype in (C128, C64):
        out, m_eff = gpu_expv(L, 0.5, HC_SX, 1, 0.4, bad, 0.3, 8, True, dtype)
        assert m_eff == 1 and np.isnan(out).all()


@pytest.mark.parametrize("L,K,m", [(6, 3, 10), (7, 3, 10), (9, 3, 10), (10, 3, 10), (13, 3, 10),
                                   (12, 4, 10), (6, 3, 16), (5, 0, 4), (13, 5, 10), (13, 5, 11)])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_reduced_basis_matches_oracle(L, K, m, dtype):
    """The paper's task sizes (dim 10, 19, 44, 60, 146) and D = 255, in the
    reduced basis, including m beyond the dimension and dim = 1.  D = 651
    (L=13, K=5) in complex128 puts the stored basis and the neighbour lists
    (4 L D bytes) just inside the 140 KiB of LDS at m = 10 and past it at
    m = 11, where each step forms the neighbours' ranks from the tables."""
    t = workloads.pe_task(L, K, 1)
    ch = pe.PEChain(t.L, t.K, t.J, t.Delta, t.hc_sites)
    assert fits(ch.dim, m, dtype)
    x = workloads.random_state(np.random.default_rng(L * 7 + K), ch.dim)
    u, tt = -0.3, 0.5
    ref, lz = krylov.expv(lambda v: ch.apply(u, v), x, tt, m, True, krylov.default_tol(),
                          return_info=True)
    B = kg.ReducedBasis(L, K)
    h = kg.XXZ(t.L, t.J, t.Delta, _lib.KG_HC_SZ, t.hc_sites)
    m_eff = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = host(kg.krylov_expv_pe(h, B, u, tt, dev_vec(x, dtype), kg.Krylov(m), m_eff=m_eff))
    assert int(host(m_eff)[0]) == lz.m_eff
    assert rel_err(out, ref) <= (1e-12 if dtype == C128 else 1e-5)


@pytest.mark.parametrize("ckpt", [0, 5])
@pytest.mark.parametrize("dtype,tol", [(C128, 1e-10), (C64, 1e-4)])
def test_gradient_matches_oracle(ckpt, dtype, tol):
    """A whole GRAPE gradient (Algorithm 1, Eq. 5) on one-block Krylov calls,
    store-all and checkpointed (three or more segments, so the recomputation
    runs beside the costate sweep), against the oracle."""
    c = workloads._random_chain(9, L=8, Delta=0.9, N=17, dt=0.07, m=12, urange=1.2)
    ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    ref = grape.gradient(ch, c.u, c.psi0, c.target, c.dt, c.m, True, krylov.default_tol())
    h = kg.XXZ(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    u = torch.tensor(c.u, dtype=torch.float64, device="cuda")
    r = kg.grape_gradient(h, u, c.dt, kg.Krylov(c.m), dev_vec(c.psi0, dtype),
                          dev_vec(c.target, dtype), ckpt_every=ckpt)
    assert abs(float(host(r.F)) - ref.F) / ref.F <= tol
    assert rel_err(host(r.grad), ref.grad) <= tol
