"""The reduced basis (fixed excitation number, even mirror parity; Sec. III.A) on
the GPU: xxz_pe_apply, krylov_expv_pe and grape_gradient_pe (all four gradient
variants) against the oracle's reduced chain (oracle/pe.py), the paper's task
sizes, and the full-size transport task (L=25, K=12) against the full-space path
on the embedded states."""

import numpy as np
import pytest
import torch

import paper_2010_03598_amd as kg
import workloads
from oracle import exact, grape, krylov, pe
from paper_2010_03598_amd import _lib
from tests.gpu_util import C64, C128, dev_vec, host, rel_err

pytestmark = pytest.mark.gpu

TOL = {C128: 1e-10, C64: 1e-4}


def xxz(t):
    return kg.XXZ(t.L, t.J, t.Delta, _lib.KG_HC_SZ, t.hc_sites)


def rand_vec(seed, dim):
    return workloads.random_state(np.random.default_rng(seed), dim)


def oracle_chain(t):
    return pe.PEChain(t.L, t.K, t.J, t.Delta, t.hc_sites)


@pytest.fixture(params=["table", "ranks"])
def gather(request, monkeypatch):
    """Both forms of the reduced H v: through the basis's neighbour table, and
    forming the neighbours' ranks in the kernel (KG_PE_NO_NEIGHBORS=1)."""
    if request.param == "ranks":
        monkeypatch.setenv("KG_PE_NO_NEIGHBORS", "1")
    else:
        monkeypatch.delenv("KG_PE_NO_NEIGHBORS", raising=False)
    return request.param


def task_vectors(t, B):
    e1 = np.zeros(B.dim, dtype=np.complex128)
    eD = np.zeros(B.dim, dtype=np.complex128)
    e1[B.index(np.array([t.e1_state]))[0]] = 1.0
    eD[B.index(np.array([t.eD_state]))[0]] = 1.0
    return e1, eD


@pytest.mark.parametrize("L,K", [(6, 3), (7, 3), (10, 3), (13, 3), (14, 7), (16, 8), (17, 6)])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_apply_vs_oracle(L, K, dtype, gather):
    t = workloads.pe_task(L, K, 1)
    ch = oracle_chain(t)
    x = rand_vec(L * 100 + K, ch.dim)
    u = 0.37
    ref = ch.apply(u, x)
    B = kg.ReducedBasis(L, K)
    assert B.dim == ch.dim
    y = host(kg.xxz_pe_apply(xxz(t), B, u, dev_vec(x, dtype)))
    tol = 1e-14 if dtype == C128 else 1e-6
    assert np.abs(y - ref).max() <= tol * np.abs(ref).max()


def test_apply_full_size_sampled(gather):
    """L=25, K=12 (2,600,612 amplitudes): sampled rows against the oracle."""
    t = workloads.pe_large()
    Bo = pe.PEBasis(t.L, t.K)
    x = rand_vec(11, Bo.dim)
    B = kg.ReducedBasis(t.L, t.K)
    u = -0.61
    y = host(kg.xxz_pe_apply(xxz(t), B, u, dev_vec(x)))
    rng = np.random.default_rng(12)
    rows = np.concatenate([[0, 1, Bo.dim - 1], rng.choice(Bo.dim, 400, replace=False)])
    ref = pe.apply_h_pe_rows(Bo, t.J, t.Delta, t.hc_sites, u, x, rows)
    assert np.abs(y[rows] - ref).max() <= 1e-14 * np.abs(ref).max()
    y64 = host(kg.xxz_pe_apply(xxz(t), B, u, dev_vec(x, C64)))
    assert np.abs(y64[rows] - ref).max() <= 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("L,K", [(25, 12), (17, 6), (28, 2)])
def test_gather_forms_agree_bit_for_bit(L, K, monkeypatch):
    """The neighbour table lists a row's bonds in ascending order, so both forms
    add the same terms in the same order: equal outputs, in both precisions."""
    t = workloads.pe_task(L, K, 1)
    B = kg.ReducedBasis(L, K)
    assert "neighbors" in kg.pe_tables_host(L, K) or L > 28
    x = rand_vec(L * 7 + K, B.dim)
    for dtype in (C128, C64):
        xd = dev_vec(x, dtype)
        monkeypatch.delenv("KG_PE_NO_NEIGHBORS", raising=False)
        y_tab = host(kg.xxz_pe_apply(xxz(t), B, 0.29, xd))
        monkeypatch.setenv("KG_PE_NO_NEIGHBORS", "1")
        y_rk = host(kg.xxz_pe_apply(xxz(t), B, 0.29, xd))
        assert np.array_equal(y_tab, y_rk)
        assert np.isfinite(y_tab).all()


@pytest.mark.parametrize("L,K,m", [(10, 3, 10), (13, 3, 10), (16, 8, 12), (6, 3, 16), (5, 0, 4)])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_krylov_vs_oracle(L, K, m, dtype, gather):
    """Including m beyond the dimension (breakdown: m_eff = dim) and dim = 1."""
    t = workloads.pe_task(L, K, 1)
    ch = oracle_chain(t)
    x = rand_vec(7 + L, ch.dim)
    u, tt = 0.2, 0.5
    ref, lz = krylov.expv(lambda v: ch.apply(u, v), x, tt, m, True, krylov.default_tol(),
                          return_info=True)
    B = kg.ReducedBasis(L, K)
    m_eff = torch.zeros(1, dtype=torch.int32, device="cuda")
    v = dev_vec(x, dtype)
    out = host(kg.krylov_expv_pe(xxz(t), B, u, tt, v, kg.Krylov(m), m_eff=m_eff))
    assert rel_err(out, ref) <= TOL[dtype]
    assert int(host(m_eff)[0]) == lz.m_eff
    if ch.dim < m:
        assert lz.m_eff == ch.dim
    # in place
    kg.krylov_expv_pe(xxz(t), B, u, tt, v, kg.Krylov(m), out=v)
    assert np.array_equal(host(v), out)


def oracle_gradient(ch, t, e1, eD, variant, nodes=3):
    if variant == "zeroth":
        return grape.gradient(ch, t.u, e1, eD, t.dt, t.m, True, krylov.default_tol())
    if variant == "centred":
        return grape.gradient_centred(ch, t.u, e1, eD, t.dt, t.m, True, krylov.default_tol())
    if variant == "first_order":
        return grape.gradient_hierarchy(ch, t.u, e1, eD, t.dt, t.m, 1, True, krylov.default_tol())
    F, g = exact.exact_gradient_quadrature(ch, t.u, e1, eD, t.dt, t.m, nodes=nodes)
    return type("R", (), {"F": F, "grad": np.array([g[j] for j in range(t.N)])})


@pytest.mark.parametrize("variant", ["zeroth", "centred", "first_order", "quadrature"])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_gradient_variants_vs_oracle(variant, dtype, gather):
    """The paper's task at D = 44 with M = 4D = 176 slices, dt = 0.5, m = 10."""
    t = workloads.pe_paper(9, 3)
    ch = oracle_chain(t)
    e1, eD = task_vectors(t, ch.B)
    ref = oracle_gradient(ch, t, e1, eD, variant)
    B = kg.ReducedBasis(t.L, t.K)
    u = torch.tensor(t.u, dtype=torch.float64, device="cuda")
    r = kg.grape_gradient_pe(xxz(t), B, u, t.dt, kg.Krylov(t.m), dev_vec(e1, dtype),
                             dev_vec(eD, dtype), variant=variant,
                             nodes=3 if variant == "quadrature" else 0)
    assert abs(float(host(r.F)) - ref.F) <= TOL[dtype] * max(ref.F, 1e-3)
    assert rel_err(host(r.grad), ref.grad) <= TOL[dtype]


@pytest.mark.parametrize("LK", sorted(workloads.PAPER_PE_DIMS))
def test_paper_sizes_forward_and_gradient(LK):
    """Every task size of Sec. III.B at its own slice count M = 4D."""
    t = workloads.pe_paper(*LK)
    ch = oracle_chain(t)
    e1, eD = task_vectors(t, ch.B)
    ref = grape.gradient(ch, t.u, e1, eD, t.dt, t.m, True, krylov.default_tol())
    B = kg.ReducedBasis(*LK)
    assert B.dim == workloads.PAPER_PE_DIMS[LK]
    u = torch.tensor(t.u, dtype=torch.float64, device="cuda")
    r = kg.grape_gradient_pe(xxz(t), B, u, t.dt, kg.Krylov(t.m), dev_vec(e1), dev_vec(eD))
    assert abs(float(host(r.F)) - ref.F) <= 1e-10 * max(ref.F, 1e-3)
    assert rel_err(host(r.grad), ref.grad) <= 1e-10


@pytest.mark.parametrize("ckpt", [1, 7, 20])
def test_checkpointing_and_states_reuse(ckpt):
    t = workloads.pe_task(14, 7, 40, seed=8)
    x0, x1 = rand_vec(1, kg.pe_dim(14, 7)), rand_vec(2, kg.pe_dim(14, 7))
    B = kg.ReducedBasis(t.L, t.K)
    h, k = xxz(t), kg.Krylov(t.m)
    u = torch.tensor(t.u, dtype=torch.float64, device="cuda")
    psi0, f = dev_vec(x0, C64), dev_vec(x1, C64)
    ref = kg.grape_gradient_pe(h, B, u, t.dt, k, psi0, f)
    r = kg.grape_gradient_pe(h, B, u, t.dt, k, psi0, f, ckpt_every=ckpt)
    assert np.array_equal(host(r.grad), host(ref.grad))
    fw = kg.grape_forward_pe(h, B, u, t.dt, k, psi0, f, ckpt_every=ckpt)
    r2 = kg.grape_gradient_pe(h, B, u, t.dt, k, psi0, f, ckpt_every=ckpt, states=fw.states,
                              states_valid=True, beta=fw.beta)
    assert np.array_equal(host(r2.grad), host(ref.grad))
    assert float(host(fw.F)) == float(host(ref.F))


def test_full_size_equals_full_space():
    """L=25, K=12 on 20 slices: the reduced-basis gradient equals the full-space
    gradient (2^25 amplitudes) of the embedded states, in FP64 and mixed precision."""
    t = workloads.pe_task(25, 12, 20, seed=6)
    Bo = pe.PEBasis(t.L, t.K)
    x0, x1 = rand_vec(21, Bo.dim), rand_vec(22, Bo.dim)
    u = torch.tensor(t.u, dtype=torch.float64, device="cuda")
    k = kg.Krylov(t.m)
    hf = kg.XXZ(t.L, t.J, t.Delta, _lib.KG_HC_SZ, t.hc_sites)
    full = kg.grape_gradient(hf, u, t.dt, k, dev_vec(Bo.embed(x0)), dev_vec(Bo.embed(x1)),
                             ckpt_every=5)
    gf, Ff = host(full.grad), float(host(full.F))
    del full
    torch.cuda.empty_cache()
    B = kg.ReducedBasis(t.L, t.K)
    for dtype in (C128, C64):
        r = kg.grape_gradient_pe(xxz(t), B, u, t.dt, k, dev_vec(x0, dtype), dev_vec(x1, dtype))
        assert abs(float(host(r.F)) - Ff) <= TOL[dtype] * max(Ff, 1e-6)
        assert rel_err(host(r.grad), gf) <= TOL[dtype]


def test_full_size_mixed_vs_fp64():
    """The transport task at L=25, K=12 with N=200 slices: complex64 vectors with
    FP64 scalars against complex128."""
    t = workloads.pe_large()
    B = kg.ReducedBasis(t.L, t.K)
    tab = kg.pe_tables_host(t.L, t.K)
    e1 = np.zeros(B.dim, dtype=np.complex128)
    eD = np.zeros(B.dim, dtype=np.complex128)
    e1[np.searchsorted(tab["reps"], min(t.e1_state, pe.reverse_bits(np.array([t.e1_state]), t.L)[0]))] = 1.0
    eD[np.searchsorted(tab["reps"], min(t.eD_state, pe.reverse_bits(np.array([t.eD_state]), t.L)[0]))] = 1.0
    u = torch.tensor(t.u, dtype=torch.float64, device="cuda")
    k = kg.Krylov(t.m)
    r128 = kg.grape_gradient_pe(xxz(t), B, u, t.dt, k, dev_vec(e1), dev_vec(eD), ckpt_every=14,
                                variant="centred")
    r64 = kg.grape_gradient_pe(xxz(t), B, u, t.dt, k, dev_vec(e1, C64), dev_vec(eD, C64),
                               ckpt_every=14, variant="centred")
    g128, g64 = host(r128.grad), host(r64.grad)
    F128, F64 = float(host(r128.F)), float(host(r64.F))
    print(f"pe_large: F = {F128:.6e}, |g| = {np.linalg.norm(g128):.3e}, mixed vs FP64: "
          f"F {abs(F64 - F128) / F128:.2e}, grad {rel_err(g64, g128):.2e}")
    assert F128 > 0.0
    assert abs(F64 - F128) <= 1e-4 * F128
    assert rel_err(g64, g128) <= 1e-4


class BruteBasis:
    """The orbit basis of a small sector of a long chain, from combinations of
    zero positions (the oracle's PEBasis enumerates all 2^L states, too many at
    L = 32); same attributes as PEBasis for the oracle's reduced H v."""

    def __init__(self, L, K):
        from itertools import combinations
        full = (1 << L) - 1
        states = sorted(full & ~sum(1 << z for z in zs) for zs in combinations(range(L), K))
        rev = lambda s: int(format(s, f"0{L}b")[::-1], 2)
        self.L, self.K = L, K
        self.reps = np.array([s for s in states if s <= rev(s)], dtype=np.int64)
        self.n = np.array([1 if rev(int(r)) == int(r) else 2 for r in self.reps])
        self.dim = self.reps.size
        self._pos = {int(r): i for i, r in enumerate(self.reps)}
        self._rev = rev

    def index(self, s):
        s = np.asarray(s, dtype=np.int64)
        return np.array([self._pos[min(int(v), self._rev(int(v)))] for v in s.ravel()],
                        dtype=np.int64).reshape(s.shape)


@pytest.mark.parametrize("L,K", [(32, 2), (31, 3), (32, 1)])
def test_apply_at_the_largest_chains(L, K, gather):
    Bo = BruteBasis(L, K)
    sites = 1 | (1 << (L - 1))
    x = rand_vec(L + K, Bo.dim)
    ref = pe.apply_h_pe(Bo, 2.0, 0.5, sites, -0.4, x)
    B = kg.ReducedBasis(L, K)
    assert B.dim == Bo.dim
    y = host(kg.xxz_pe_apply(kg.XXZ(L, 2.0, 0.5, _lib.KG_HC_SZ, sites), B, -0.4, dev_vec(x)))
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()


def test_gradient_at_L32():
    """Zeroth-order gradient of a random transfer in the (32, 2) sector vs the oracle's
    sweeps on the reduced chain."""
    L, K, N, dt, m = 32, 2, 12, 0.3, 12
    Bo = BruteBasis(L, K)
    sites = 1 | (1 << (L - 1))

    class Chain:
        def apply(self, u, v):
            return pe.apply_h_pe(Bo, 2.0, 0.5, sites, u, v)

        def apply_hc(self, v):
            from oracle import model
            return model.sz_control_diag(L, sites, Bo.reps).real * v

    rng = np.random.default_rng(4)
    u = rng.uniform(-1, 1, N)
    x0, x1 = rand_vec(5, Bo.dim), rand_vec(6, Bo.dim)
    ref = grape.gradient(Chain(), u, x0, x1, dt, m, True, krylov.default_tol())
    B = kg.ReducedBasis(L, K)
    r = kg.grape_gradient_pe(kg.XXZ(L, 2.0, 0.5, _lib.KG_HC_SZ, sites), B,
                             torch.tensor(u, device="cuda"), dt, kg.Krylov(m), dev_vec(x0),
                             dev_vec(x1), ckpt_every=4)
    assert abs(float(host(r.F)) - ref.F) <= 1e-10 * ref.F
    assert rel_err(host(r.grad), ref.grad) <= 1e-10
